// Host side of libwqa: the C ABI declared in include/wqa.h.
//
// Responsibilities (all setup, none of it on the timed path):
//   * the spline space: open knots per direction, uniform by default or with given
//     breakpoints (Sec. 2.2, eq:Gmap3, eq:DimUni);
//   * the weighted Gaussian rules: Newton in x87 extended precision on the exactness conditions
//     (eq:GaussQuadSys / eq:GaussQuadSysStiff) for the paper's interior rules
//     (Sec. 3.1.1, 3.1.2, 3.2.1, 3.2.2) and for the boundary rows the paper leaves
//     open (Remark closing Sec. 3.2); on non-uniform knots, the same rules traced from
//     the uniform ones by homotopy continuation of the knot vector (the approach the
//     paper names for its future work, Sec. 1 and Conclusion);
//   * validation of caller-supplied rules (exactness against element-wise
//     Gauss-Legendre integrals, nodes inside the support and off the knots);
//   * contraction tables T[j][q][s] = w * phi_j(x) * phi_{j-p+s}(x) per direction and
//     kind, the factors of the sum-factorized integrand (eq:Decompo), in FP64 with
//     an FP32 copy rounded from them, uploaded once to the device;
//   * argument checks and kernel dispatch for the assemble calls.
#include "wqa.h"
#include "wqa_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <thread>
#include <vector>

namespace {

thread_local std::string g_error;

wqa_status fail(wqa_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return st;
}

wqa_status ok() {
    g_error.clear();
    return WQA_OK;
}

// ---------------------------------------------------------------------------------
// The rule solver, the basis and the table builder work in x87 extended precision
// (64-bit significand), so that the FP64 rules and tables they produce are correctly
// rounded up to the conditioning of the exactness systems.
using real = long double;
constexpr real PI = 3.141592653589793238462643383279502884L;

// B-splines on an open knot vector in element units: knot t_i = b[clamp(i - p, 0, nel)]
// with breakpoints b (b_e = e for uniform knots, b == nullptr).  Cox-de Boor with
// right-continuous degree-0 pieces, the last interval closed at the right end.
struct Knots {
    int p;
    int64_t nel;
    const real *b = nullptr;      // nel + 1 breakpoints in element units, or nullptr: uniform
    real t(int64_t i) const {
        int64_t v = i - p;
        v = v < 0 ? 0 : (v > nel ? nel : v);
        return b ? b[v] : (real)v;
    }
    real brk(int64_t e) const { return t(e + p); }      // left end of element e
};

real bspline(const Knots &kn, int64_t i, int deg, real u) {
    real v[8];
    const real last = kn.brk(kn.nel);
    for (int k = 0; k <= deg; ++k) {
        real a = kn.t(i + k), b = kn.t(i + k + 1);
        bool in = (a <= u && u < b) || (u == last && b == last && a < b);
        v[k] = in ? 1.0 : 0.0;
    }
    for (int r = 1; r <= deg; ++r) {
        for (int k = 0; k + r <= deg; ++k) {
            int64_t ii = i + k;
            real term = 0.0;
            real d1 = kn.t(ii + r) - kn.t(ii);
            if (d1 != 0.0) term += (u - kn.t(ii)) / d1 * v[k];
            real d2 = kn.t(ii + r + 1) - kn.t(ii + 1);
            if (d2 != 0.0) term += (kn.t(ii + r + 1) - u) / d2 * v[k + 1];
            v[k] = term;
        }
    }
    return v[0];
}

// d/du B_{i,p}(u), element units.
real bspline_du(const Knots &kn, int64_t i, int p, real u) {
    real out = 0.0;
    real d1 = kn.t(i + p) - kn.t(i);
    if (d1 != 0.0) out += p / d1 * bspline(kn, i, p - 1, u);
    real d2 = kn.t(i + p + 1) - kn.t(i + 1);
    if (d2 != 0.0) out -= p / d2 * bspline(kn, i + 1, p - 1, u);
    return out;
}

real phi(const Knots &kn, int kind, int64_t i, real u) {
    return kind == WQA_MASS ? bspline(kn, i, kn.p, u) : bspline_du(kn, i, kn.p, u);
}

// m-point Gauss-Legendre on [0, 1] (Newton on the Legendre recurrence).
void gauss_legendre(int m, std::vector<real> &x, std::vector<real> &w) {
    x.assign(m, 0.0);
    w.assign(m, 0.0);
    for (int k = 0; k < m; ++k) {
        real y = std::cos(PI * (k + 0.75) / (m + 0.5));
        real dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            real p0 = 1.0, p1 = y;
            for (int n = 2; n <= m; ++n) {
                real p2 = ((2 * n - 1) * y * p1 - (n - 1) * p0) / n;
                p0 = p1;
                p1 = p2;
            }
            dp = m * (y * p1 - p0) / (y * y - 1.0);
            real dy = p1 / dp;
            y -= dy;
            if (std::fabs(dy) < 1e-19L) break;
        }
        real p0 = 1.0, p1 = y;
        for (int n = 2; n <= m; ++n) {
            real p2 = ((2 * n - 1) * y * p1 - (n - 1) * p0) / n;
            p0 = p1;
            p1 = p2;
        }
        dp = m * (y * p1 - p0) / (y * y - 1.0);
        x[k] = (1.0 - y) / 2.0;
        w[k] = 1.0 / ((1.0 - y * y) * dp * dp);
    }
}

// Integral of f (element units) over elements lo .. hi-1 of the knots, m-point
// Gauss-Legendre per element: exact for piecewise polynomials of degree <= 2m - 1 with
// breakpoints at the knots.
template <class F>
real integrate(F f, const Knots &kn, int64_t lo, int64_t hi, int m) {
    // the m-point rule, computed once per m and thread (validation calls this per row)
    thread_local std::vector<real> rule_x[16], rule_w[16];
    if (m < 1 || m >= 16) std::abort();
    if (rule_x[m].empty()) gauss_legendre(m, rule_x[m], rule_w[m]);
    const std::vector<real> &gx = rule_x[m], &gw = rule_w[m];
    real s = 0.0;
    for (int64_t e = lo; e < hi; ++e) {
        const real a = kn.brk(e), L = kn.brk(e + 1) - a;
        for (int k = 0; k < m; ++k) s += gw[k] * L * f(a + L * gx[k]);
    }
    return s;
}

// ---------------------------------------------------------------------------------
// Newton-Raphson for a small square system, central-difference Jacobian, partial
// pivoting.  Returns false on a singular step or when the residual does not fall
// below tol within the step budget.
template <class F>
bool newton(F residual, std::vector<real> &v, real tol) {
    const int n = (int)v.size();
    std::vector<real> f(n), fp(n), fm(n), J(n * n), dx(n);
    for (int it = 0; it < 80; ++it) {
        residual(v, f);
        real nf = 0.0;
        for (real e : f) nf = std::max(nf, std::fabs(e));
        if (!std::isfinite(nf)) return false;
        for (int c = 0; c < n; ++c) {
            real h = (real)1e-6 * std::max((real)1, std::fabs(v[c]));
            std::vector<real> vp = v, vm = v;
            vp[c] += h;
            vm[c] -= h;
            residual(vp, fp);
            residual(vm, fm);
            for (int r = 0; r < n; ++r) J[r * n + c] = (fp[r] - fm[r]) / (2 * h);
        }
        // solve J dx = f
        std::vector<real> A = J, b = f;
        for (int c = 0; c < n; ++c) {
            int piv = c;
            for (int r = c + 1; r < n; ++r)
                if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
            if (std::fabs(A[piv * n + c]) < 1e-300L) return false;
            if (piv != c) {
                for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
                std::swap(b[c], b[piv]);
            }
            for (int r = c + 1; r < n; ++r) {
                real m = A[r * n + c] / A[c * n + c];
                for (int k = c; k < n; ++k) A[r * n + k] -= m * A[c * n + k];
                b[r] -= m * b[c];
            }
        }
        for (int c = n - 1; c >= 0; --c) {
            real s = b[c];
            for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * dx[k];
            dx[c] = s / A[c * n + c];
        }
        real step = 0.0;
        for (int k = 0; k < n; ++k) {
            v[k] -= dx[k];
            step = std::max(step, std::fabs(dx[k]));
            if (!std::isfinite(v[k]) || std::fabs(v[k]) > 1e6) return false;
        }
        if (nf < tol && step < 1e-18L) return true;
    }
    residual(v, f);
    real nf = 0.0;
    for (real e : f) nf = std::max(nf, std::fabs(e));
    return nf < tol;
}

// A rule in element units for one row: nodes tau, weights omega (multiplying phi_i phi_j).
struct LocalRule {
    std::vector<real> tau, omega;
};

// Cardinal interior rule of the paper for (p, kind), parametrized as in Sec. 3:
// symmetric about (p+1)/2; p = 2 with middle node 3/2 (and, for stiffness, middle
// weight 8/9 which multiplies B'_j(3/2) = 0); p = 3 stiffness with omega_1 = 1 and
// the smaller of the two admissible tau_1.
bool solve_interior(int p, int kind, LocalRule &out) {
    const Knots kn{p, 4 * p + 4};
    const int64_t j = 2 * p + 1, base = j - p;
    const real half = 0.5 * (p + 1);
    auto expand = [&](const std::vector<real> &v, LocalRule &r) {
        if (p == 2) {
            real t1 = v[0];
            r.tau = {t1, half, 2 * half - t1};
            if (kind == WQA_MASS) r.omega = {v[1], v[2], v[1]};
            else r.omega = {v[1], 8.0 / 9.0, v[1]};
        } else {
            real t1 = v[0], t2 = v[1];
            r.tau = {t1, t2, 2 * half - t2, 2 * half - t1};
            if (kind == WQA_MASS) r.omega = {v[2], v[3], v[3], v[2]};
            else r.omega = {1.0, v[2], v[2], 1.0};
        }
    };
    const int nu = (p == 2) ? (kind == WQA_MASS ? 3 : 2) : (kind == WQA_MASS ? 4 : 3);
    // exactness against columns j, j+1, ..., j+nu-1 (the mirrored columns follow by symmetry)
    std::vector<real> exact(nu);
    for (int o = 0; o < nu; ++o)
        exact[o] = integrate([&](real u) { return phi(kn, kind, j + o, u) * phi(kn, kind, j, u); }, kn,
                             base, j + 1, p + 2);
    auto residual = [&](const std::vector<real> &v, std::vector<real> &f) {
        LocalRule r;
        expand(v, r);
        for (int o = 0; o < nu; ++o) {
            real s = 0.0;
            for (size_t q = 0; q < r.tau.size(); ++q) {
                real u = base + r.tau[q];
                s += r.omega[q] * phi(kn, kind, j + o, u) * phi(kn, kind, j, u);
            }
            f[o] = s - exact[o];
        }
    };
    auto admissible = [&](const std::vector<real> &v) {
        LocalRule r;
        expand(v, r);
        for (int q = 0; q <= p; ++q)
            if (!(r.tau[q] > q && r.tau[q] < q + 1)) return false;
        for (real w : r.omega)
            if (!(w > 0)) return false;
        if (p == 3 && kind == WQA_STIFFNESS && !(r.tau[0] < 0.5)) return false;
        return true;
    };
    const real offs[] = {0.25, 0.5, 0.75, 0.4};
    const real ws[] = {1.0, 0.5};
    for (real off : offs)
        for (real w : ws) {
            std::vector<real> v;
            if (p == 2) v = (kind == WQA_MASS) ? std::vector<real>{off, w, w} : std::vector<real>{off, w};
            else v = (kind == WQA_MASS) ? std::vector<real>{off, 1 + off, w, w}
                                        : std::vector<real>{off, 1 + off, w};
            if (newton(residual, v, (real)1e-18L) && admissible(v)) {
                expand(v, out);
                return true;
            }
        }
    return false;
}

// Node count and number of extra conditions for left boundary row j < p; the extra
// functions are x^{deg+1}, (x-1)_+^{deg+1}, ... with deg = p (mass) or p-1 (stiffness).
// Node count ceil(m/2) for m independent exactness conditions, except cubic
// stiffness row 1 whose square 2-node system has no real root.
void boundary_shape(int p, int kind, int j, int &n, int &extra) {
    static const int tab[2][2][3][2] = {
        // mass: p = 2 rows 0,1 ; p = 3 rows 0,1,2
        {{{2, 1}, {2, 0}, {0, 0}}, {{2, 0}, {3, 1}, {3, 0}}},
        // stiffness
        {{{1, 0}, {2, 1}, {0, 0}}, {{2, 1}, {3, 2}, {3, 1}}},
    };
    n = tab[kind][p - 2][j][0];
    extra = tab[kind][p - 2][j][1];
}

bool solve_boundary(int p, int kind, int j, LocalRule &out) {
    const Knots kn{p, 4 * p + 4};
    int n, n_extra;
    boundary_shape(p, kind, j, n, n_extra);
    const int deg = (kind == WQA_MASS) ? p : p - 1;
    int n_cols = j + p + 1 - (kind == WQA_STIFFNESS ? 1 : 0);   // sum_i B'_i = 0 drops one
    const int m = n_cols + n_extra;
    if (m != 2 * n) return false;
    auto test = [&](int t, real u) {
        if (t < n_cols) return phi(kn, kind, t, u);
        real y = u - (t - n_cols);
        return y > 0 ? std::pow(y, (real)(deg + 1)) : (real)0;
    };
    std::vector<real> exact(m);
    for (int t = 0; t < m; ++t)
        exact[t] = integrate([&](real u) { return test(t, u) * phi(kn, kind, j, u); }, kn, 0, j + 1, p + 3);
    auto residual = [&](const std::vector<real> &v, std::vector<real> &f) {
        for (int t = 0; t < m; ++t) {
            real s = 0.0;
            for (int q = 0; q < n; ++q) s += v[n + q] * test(t, v[q]) * phi(kn, kind, j, v[q]);
            f[t] = s - exact[t];
        }
    };
    auto admissible = [&](const std::vector<real> &v) {
        for (int q = 0; q < n; ++q) {
            real t = v[q];
            if (!(t > 0 && t < j + 1)) return false;
            if (std::fabs(t - std::nearbyint(t)) < 1e-8L) return false;
            if (q + 1 < n && !(t < v[q + 1])) return false;
            if (!(v[n + q] > 0)) return false;
        }
        return true;
    };
    const real L = j + 1;
    const real shifts[] = {0.5, 0.25, 0.75, 1.0 / 3, 2.0 / 3};
    const real spreads[] = {1.0, 0.75};
    const real ws[] = {0.5, 1.0};
    for (real sh : shifts)
        for (real sp : spreads)
            for (real w : ws) {
                std::vector<real> v(2 * n);
                for (int q = 0; q < n; ++q) {
                    v[q] = L * (q + sh) / n * sp + L * (1 - sp) / 2;
                    v[n + q] = w;
                }
                if (newton(residual, v, (real)1e-18L) && admissible(v)) {
                    out.tau.assign(v.begin(), v.begin() + n);
                    out.omega.assign(v.begin() + n, v.end());
                    return true;
                }
            }
    return false;
}

// ---------------------------------------------------------------------------------
// Rules on non-uniform knots.  Each row's rule is traced from its uniform rule along the
// straight path of the breakpoints, b(lam) = (1 - lam) b_uniform + lam b_target (element
// units, uniform b_e = e), with Newton at every step starting from the previous root.
// On uniform knots the interior rules fix their free parameter by symmetry; off them,
// the condition symmetry leaves in each element's own coordinate
// r = (x - b_e) / (b_{e+1} - b_e) of the node's element takes its place:
//   quadratic mass: the middle node at r = 1/2 (the paper's tau_2 = 3/2);
//   cubic mass and stiffness: r(first node) + r(last node) = 1; cubic stiffness also
//     keeps omega_1 equal to the length of the support's first element (1 on uniform
//     knots, the paper's choice);
//   quadratic stiffness: the middle node at the zero of B'_j in the middle element
//     (3/2 on uniform knots), with the printed weight 8/9 (it multiplies 0).
// Boundary rows keep their square systems with the actual knots (the extra functions
// are truncated powers at the first distinct knots from the clamped end).  A path that
// runs into a singular point (a stiffness node meeting the zero of B'_j, where its weight
// diverges) has no rule of this family at its end: the solver reports failure.
struct RowSystem {
    int p, kind;
    int64_t j, n;
    bool interior;
    int nn = 0;                                  // boundary rows: node count
    Knots kn{0, 0, nullptr};
    real mid = 0;                                // quadratic stiffness: the middle node
    std::vector<std::function<real(real)>> tests;
    std::vector<real> exact;

    RowSystem(int p_, int kind_, int64_t j_, int64_t n_)
        : p(p_), kind(kind_), j(j_), n(n_), interior(j_ >= p_ && j_ < n_ - p_) {}

    real lo(int q) const { return kn.t(j + q); }          // left end of support element q
    real rel(int q, real x) const { return (x - lo(q)) / (lo(q + 1) - lo(q)); }

    void setup(const Knots &k) {
        kn = k;
        tests.clear();
        auto column = [this](int64_t i) { return [this, i](real u) { return phi(kn, kind, i, u); }; };
        if (interior) {
            const int64_t last = (kind == WQA_MASS) ? j + p : j + p - 1;   // sum_i B'_i = 0 drops one
            for (int64_t i = j - p; i <= last; ++i) tests.push_back(column(i));
            if (kind == WQA_STIFFNESS && p == 2) {
                const real a = lo(1), b = lo(2);                  // B'_j is linear there
                const real da = phi(kn, kind, j, a), db = phi(kn, kind, j, b);
                mid = a + da * (b - a) / (da - db);
            }
        } else {
            const bool left = j < p;
            int extra = 0;
            boundary_shape(p, kind, (int)(left ? j : n - 1 - j), nn, extra);
            const int deg = (kind == WQA_MASS) ? p : p - 1;
            int64_t first = left ? 0 : j - p, last = left ? j + p : n - 1;
            if (kind == WQA_STIFFNESS) {
                if (left) --last;
                else ++first;
            }
            for (int64_t i = first; i <= last; ++i) tests.push_back(column(i));
            for (int k2 = 0; k2 < extra; ++k2) {
                if (left) {
                    const real t = kn.brk(k2);
                    tests.push_back([t, deg](real u) { return u > t ? std::pow(u - t, (real)(deg + 1)) : (real)0; });
                } else {
                    const real t = kn.brk(kn.nel - k2);
                    tests.push_back([t, deg](real u) { return u < t ? std::pow(t - u, (real)(deg + 1)) : (real)0; });
                }
            }
        }
        exact.assign(tests.size(), 0);
        const int64_t e_lo = std::max<int64_t>(0, j - p), e_hi = std::min<int64_t>(kn.nel, j + 1);
        for (size_t t = 0; t < tests.size(); ++t)
            exact[t] = integrate([&](real u) { return tests[t](u) * phi(kn, kind, j, u); }, kn, e_lo, e_hi, 2 * p + 2);
    }

    void expand(const std::vector<real> &v, std::vector<real> &tau, std::vector<real> &om) const {
        if (!interior) {
            tau.assign(v.begin(), v.begin() + nn);
            om.assign(v.begin() + nn, v.end());
        } else if (kind == WQA_MASS && p == 2) {
            tau = {v[0], (lo(1) + lo(2)) / 2, v[1]};
            om = {v[2], v[3], v[4]};
        } else if (kind == WQA_MASS) {
            tau.assign(v.begin(), v.begin() + 4);
            om.assign(v.begin() + 4, v.end());
        } else if (p == 2) {
            tau = {v[0], mid, v[1]};
            om = {v[2], (real)8 / 9, v[3]};
        } else {
            tau.assign(v.begin(), v.begin() + 4);
            om = {lo(1) - lo(0), v[4], v[5], v[6]};
        }
    }

    std::vector<real> unknowns(const std::vector<real> &tau, const std::vector<real> &om) const {
        if (!interior || (kind == WQA_MASS && p == 3)) {
            std::vector<real> v(tau);
            v.insert(v.end(), om.begin(), om.end());
            return v;
        }
        if (kind == WQA_MASS) return {tau[0], tau[2], om[0], om[1], om[2]};
        if (p == 2) return {tau[0], tau[2], om[0], om[2]};
        return {tau[0], tau[1], tau[2], tau[3], om[1], om[2], om[3]};
    }

    void residual(const std::vector<real> &v, std::vector<real> &f) const {
        std::vector<real> tau, om;
        expand(v, tau, om);
        f.assign(v.size(), 0);
        for (size_t t = 0; t < tests.size(); ++t) {
            real sum = 0;
            for (size_t q = 0; q < tau.size(); ++q) sum += om[q] * phi(kn, kind, j, tau[q]) * tests[t](tau[q]);
            f[t] = sum - exact[t];
        }
        if (interior && p == 3) f[tests.size()] = rel(0, tau[0]) + rel(3, tau[3]) - 1;
    }

    bool admissible(const std::vector<real> &v) const {
        std::vector<real> tau, om;
        expand(v, tau, om);
        for (real w : om)
            if (!(w > 0)) return false;
        if (interior) {
            for (int q = 0; q <= p; ++q)
                if (!(tau[q] > lo(q) && tau[q] < lo(q + 1))) return false;
            if (p == 3 && kind == WQA_STIFFNESS && !(tau[0] < (lo(0) + lo(1)) / 2)) return false;
            return true;
        }
        const real a = kn.t(j), b = kn.t(j + p + 1);
        for (size_t q = 0; q < tau.size(); ++q) {
            if (!(tau[q] > a && tau[q] < b)) return false;
            if (q + 1 < tau.size() && !(tau[q] < tau[q + 1])) return false;
            for (int64_t e = std::max<int64_t>(0, j - p); e <= std::min<int64_t>(kn.nel - 1, j); ++e) {
                const real ea = kn.brk(e), eb = kn.brk(e + 1), tiny = (real)1e-8 * (eb - ea);
                if (std::fabs(tau[q] - ea) < tiny || std::fabs(tau[q] - eb) < tiny) return false;
            }
        }
        return true;
    }
};

// Traces row j's rule (element units, unpadded) from the uniform one to the knots with
// breakpoints `target` (element units, nel + 1 values).
bool trace_row(int p, int kind, int64_t j, int64_t nel, const std::vector<real> &target, const LocalRule &uniform,
               LocalRule &out) {
    RowSystem rs(p, kind, j, nel + p);
    // The row is solved in coordinates local to its support: every knot is taken relative
    // to the support's first breakpoint e0, all along the path (differences formed before
    // they are mixed, so nothing large cancels).  Magnitudes then stay O(p) on every row;
    // in absolute element units, rows far from the origin sit where one unit in the last
    // place of a node exceeds Newton's tolerances.  The previous root, carried in these
    // coordinates, also moves with the support from one step to the next.
    const int64_t e0 = j - p > 0 ? j - p : 0;
    std::vector<real> br(nel + 1);
    auto knots_at = [&](real lam) {
        for (int64_t e = 0; e <= nel; ++e) br[e] = (1 - lam) * (real)(e - e0) + lam * (target[e] - target[e0]);
        return Knots{p, nel, br.data()};
    };
    auto res = [&](const std::vector<real> &v, std::vector<real> &f) { rs.residual(v, f); };
    rs.setup(knots_at(0));
    std::vector<real> tau0 = uniform.tau;
    for (real &x : tau0) x -= (real)e0;
    std::vector<real> v = rs.unknowns(tau0, uniform.omega);
    real lam = 0, step = (real)0.25;
    while (lam < 1) {
        const real nxt = std::min((real)1, lam + step);
        rs.setup(knots_at(nxt));
        std::vector<real> w = v;
        if (newton(res, w, (real)1e-17L) && rs.admissible(w)) {
            v = w;
            lam = nxt;
            step = std::min(step * 2, (real)0.25);
        } else {
            step /= 2;
            if (step < (real)1 / 4096) return false;
        }
    }
    rs.expand(v, out.tau, out.omega);
    for (real &x : out.tau) x += target[e0];
    return true;
}

}  // namespace

// ---------------------------------------------------------------------------------
struct wqa_ctx {
    int device = -1;
    int dim = 0, p = 0;
    bool have_space = false;
    int64_t nel[wqa::kMaxDim] = {0, 0, 0};
    int64_t n[wqa::kMaxDim] = {0, 0, 0};
    int64_t N[wqa::kMaxDim] = {0, 0, 0};
    std::vector<real> brk[wqa::kMaxDim];      // breakpoints in element units; empty: uniform
    std::vector<double> nodes[2][wqa::kMaxDim], omega[2][wqa::kMaxDim];
    std::vector<double> tab64[2][wqa::kMaxDim];
    std::vector<float> tab32[2][wqa::kMaxDim];
    bool have_rule[2][wqa::kMaxDim] = {};
    // the rows at least p from both ends have tables that vanish outside q <= s <= q + p
    bool banded[2][wqa::kMaxDim] = {};
    int64_t max_tasks = wqa::kMaxTasksPerDispatch;      // wave tasks per kernel dispatch
    int64_t pitch = 0;                                  // grid line pitch (0: dense, N of the last direction)
    int samples = WQA_SAMPLES_GRID;                     // layout of the sample buffers
    // device copies
    void *dev = nullptr;
    size_t dev_bytes = 0;
    const float *d32[2][wqa::kMaxDim] = {};
    const double *d64[2][wqa::kMaxDim] = {};
    bool dev_current = false;
    int final_mode = WQA_FINAL_F64;
};

namespace {

int Q_of(const wqa_ctx *c) { return c->p + 1; }

Knots knots_of(const wqa_ctx *c, int dir) {
    return Knots{c->p, c->nel[dir], c->brk[dir].empty() ? nullptr : c->brk[dir].data()};
}
int S_of(const wqa_ctx *c) { return 2 * c->p + 1; }

bool rules_complete(const wqa_ctx *c) {
    for (int k = 0; k < c->dim; ++k)
        if (!c->have_rule[WQA_MASS][k] || !c->have_rule[WQA_STIFFNESS][k]) return false;
    return true;
}

// Builds T[j][q][s] = w_jq phi_j(x_jq) phi_{j-p+s}(x_jq) for one kind and direction, in
// parametric units (the stiffness factor carries nel^2 from d/dx = nel d/du).
// Host threads for setup work: OMP_NUM_THREADS when set (the process's share of the
// host), else the hardware's count; at most 64.
int64_t host_threads() {
    int64_t t = (int64_t)std::thread::hardware_concurrency();
    if (const char *env = std::getenv("OMP_NUM_THREADS")) {
        const long v = std::strtol(env, nullptr, 10);
        if (v > 0) t = v;
    }
    return std::max<int64_t>(1, std::min<int64_t>(t, 64));
}

// body(j0, j1) over the rows [0, n) in contiguous chunks of at least `grain` rows on
// host threads (a single call when one chunk remains); body must only write state of
// its own rows.
template <class F>
void for_rows(int64_t n, int64_t grain, F body) {
    const int64_t chunks = std::min<int64_t>(host_threads(), n / grain);
    if (chunks <= 1) {
        body((int64_t)0, n);
        return;
    }
    std::vector<std::thread> pool;
    for (int64_t t = 0; t < chunks; ++t) pool.emplace_back(body, n * t / chunks, n * (t + 1) / chunks);
    for (std::thread &th : pool) th.join();
}

void build_table(wqa_ctx *c, int kind, int dir) {
    const int p = c->p, Q = Q_of(c), S = S_of(c);
    const int64_t n = c->n[dir], nel = c->nel[dir];
    const Knots kn = knots_of(c, dir);
    std::vector<double> &T = c->tab64[kind][dir];
    T.assign((size_t)n * Q * S, 0.0);
    const real scale = (kind == WQA_MASS) ? (real)1 : (real)nel * (real)nel;
    std::vector<float> &T32 = c->tab32[kind][dir];
    T32.resize(T.size());
    const std::vector<double> &xs = c->nodes[kind][dir], &ws = c->omega[kind][dir];
    for_rows(n, 16384, [&](int64_t j0, int64_t j1) {
        for (int64_t j = j0; j < j1; ++j)
            for (int q = 0; q < Q; ++q) {
                const real x = xs[j * Q + q];
                const real w = ws[j * Q + q];
                const real u = x * (real)nel;
                const real own = phi(kn, kind, j, u);
                for (int s = 0; s < S; ++s) {
                    const int64_t col = j - p + s, at = (j * Q + q) * S + s;
                    if (col >= 0 && col < n && w != 0) T[at] = (double)(w * scale * own * phi(kn, kind, col, u));
                    T32[at] = (float)T[at];
                }
            }
    });
    // The kernels skip the entries outside q <= s <= q + p of rows at least p from both
    // ends; that holds when node q of each such row lies in element q of its support (the
    // library's rules), so it is checked on the built table rather than assumed.
    bool banded = true;
    for (int64_t j = p; j < n - p && banded; ++j)
        for (int q = 0; q < Q && banded; ++q)
            for (int s = 0; s < S; ++s)
                if ((s < q || s > q + p) && T[(j * Q + q) * S + s] != 0.0) {
                    banded = false;
                    break;
                }
    c->banded[kind][dir] = banded;
}

wqa_status upload(wqa_ctx *c) {
    if (c->device < 0 || c->dev_current) return WQA_OK;
    if (!rules_complete(c)) return WQA_OK;
    const int Q = Q_of(c), S = S_of(c);
    size_t need = 0;
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < c->dim; ++k) need += (size_t)c->n[k] * Q * S * (8 + 4) + 512;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return fail(WQA_EHIP, "hipSetDevice(%d): %s", c->device, hipGetErrorString(e));
    // Kernels queued earlier on any stream may still read the tables: wait for the device
    // before they are rewritten in place or freed.
    if (c->dev) {
        e = hipDeviceSynchronize();
        if (e != hipSuccess) return fail(WQA_EHIP, "waiting for queued kernels before a table upload: %s",
                                         hipGetErrorString(e));
    }
    if (need > c->dev_bytes) {
        if (c->dev) {
            (void)hipFree(c->dev);
            c->dev = nullptr;
            c->dev_bytes = 0;
        }
        e = hipMalloc(&c->dev, need);
        if (e != hipSuccess) return fail(WQA_ENOMEM, "hipMalloc(%zu) for rule tables: %s", need, hipGetErrorString(e));
        c->dev_bytes = need;
    }
    char *base = (char *)c->dev;
    size_t off = 0;
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < c->dim; ++k) {
            size_t cnt = c->tab64[r][k].size();
            off = (off + 255) & ~(size_t)255;
            e = hipMemcpy(base + off, c->tab64[r][k].data(), cnt * 8, hipMemcpyHostToDevice);
            if (e != hipSuccess) return fail(WQA_EHIP, "table upload: %s", hipGetErrorString(e));
            c->d64[r][k] = (const double *)(base + off);
            off += cnt * 8;
            off = (off + 255) & ~(size_t)255;
            e = hipMemcpy(base + off, c->tab32[r][k].data(), cnt * 4, hipMemcpyHostToDevice);
            if (e != hipSuccess) return fail(WQA_EHIP, "table upload: %s", hipGetErrorString(e));
            c->d32[r][k] = (const float *)(base + off);
            off += cnt * 4;
        }
    c->dev_current = true;
    return WQA_OK;
}

// Validation of one direction's rule (see wqa_set_rules).
// sampled: the rules are translates of one another on uniform knots (the library's own
// default rules), so beyond 4096 rows the exactness integrals are checked on the 2p+1
// rows at each end, every 97th row and the last interior row (the largest coordinates,
// hence the largest node rounding); the node checks still cover every row.
wqa_status validate(const wqa_ctx *c, int kind, int dir, const double *x, const double *w, double tol,
                    bool sampled = false) {
    const int p = c->p, Q = Q_of(c);
    const int64_t n = c->n[dir], nel = c->nel[dir];
    const Knots kn = knots_of(c, dir);
    auto integrals_checked = [&](int64_t j) {
        return !sampled || n <= 4096 || j <= 2 * p || j >= n - 2 * p - 2 || j % 97 == 0;
    };
    for (int64_t j = 0; j < n; ++j) {
        const real lo = kn.t(j), hi = kn.t(j + p + 1);
        const int64_t e_lo = std::max<int64_t>(0, j - p), e_hi = std::min<int64_t>(nel, j + 1);   // support elements
        for (int q = 0; q < Q; ++q) {
            double xv = x[j * Q + q], wv = w[j * Q + q];
            if (!std::isfinite(xv) || !std::isfinite(wv) || xv < 0.0 || xv > 1.0)
                return fail(WQA_ERULE, "row %lld node %d: x=%g w=%g outside [0,1] or not finite",
                            (long long)j, q, xv, wv);
            if (wv == 0.0) continue;
            real u = (real)xv * (real)nel;
            if (!(u > lo && u < hi))
                return fail(WQA_ERULE, "row %lld node %d at %.17g lies outside the support [%g, %g] (element units)",
                            (long long)j, q, (double)u, (double)lo, (double)hi);
            for (int64_t e = e_lo; e < e_hi; ++e) {
                const real a = kn.brk(e), b = kn.brk(e + 1), tiny = (real)1e-9 * (b - a);
                if (std::fabs(u - a) < tiny || std::fabs(u - b) < tiny)
                    return fail(WQA_ERULE, "row %lld node %d at %.17g sits on a knot", (long long)j, q, (double)u);
            }
        }
        if (tol < 0 || !integrals_checked(j)) continue;
        real worst = 0, scale = 0;
        for (int64_t i = std::max<int64_t>(0, j - p); i <= std::min<int64_t>(n - 1, j + p); ++i) {
            real exact = integrate([&](real u) { return phi(kn, kind, i, u) * phi(kn, kind, j, u); }, kn,
                                   e_lo, e_hi, p + 2);
            real quad = 0;
            for (int q = 0; q < Q; ++q) {
                real u = (real)x[j * Q + q] * (real)nel;
                quad += (real)w[j * Q + q] * (real)nel * phi(kn, kind, i, u) * phi(kn, kind, j, u);
            }
            worst = std::max(worst, std::fabs(quad - exact));
            scale = std::max(scale, std::fabs(exact));
        }
        if (worst > (real)tol * scale)
            return fail(WQA_ERULE, "%s rule of direction %d, row %lld: relative exactness residual %.3g > %.3g",
                        kind == WQA_MASS ? "mass" : "stiffness", dir, (long long)j, (double)(worst / scale), tol);
    }
    return WQA_OK;
}

wqa_status install(wqa_ctx *c, int kind, int dir, const double *x, const double *w) {
    const size_t cnt = (size_t)c->n[dir] * Q_of(c);
    c->nodes[kind][dir].assign(x, x + cnt);
    c->omega[kind][dir].assign(w, w + cnt);
    c->have_rule[kind][dir] = true;
    build_table(c, kind, dir);
    c->dev_current = false;
    return upload(c);
}

// Default rule of one direction: interior rows translate the cardinal rule, the p rows
// at each end use the boundary rules (mirrored on the right), padded with zero-weight
// nodes at the middle of the support's outermost element.
wqa_status default_direction(wqa_ctx *c, const LocalRule &interior, const std::vector<LocalRule> &boundary,
                             int dir, std::vector<double> &x, std::vector<double> &w) {
    const int p = c->p, Q = Q_of(c);
    const int64_t n = c->n[dir], nel = c->nel[dir];
    const real fn = (real)nel;
    x.assign((size_t)n * Q, 0.0);
    w.assign((size_t)n * Q, 0.0);
    for (int64_t j = 0; j < n; ++j) {
        double *xj = &x[j * Q], *wj = &w[j * Q];
        if (j >= p && j < n - p) {
            for (int q = 0; q < Q; ++q) {
                xj[q] = (double)(((real)(j - p) + interior.tau[q]) / fn);
                wj[q] = (double)(interior.omega[q] / fn);
            }
        } else if (j < p) {
            const LocalRule &b = boundary[j];
            const int m = (int)b.tau.size();
            for (int q = 0; q < Q; ++q) {
                xj[q] = (double)((q < m ? b.tau[q] : (real)0.5) / fn);
                wj[q] = q < m ? (double)(b.omega[q] / fn) : 0.0;
            }
        } else {
            const LocalRule &b = boundary[n - 1 - j];
            const int m = (int)b.tau.size();
            for (int q = 0; q < Q; ++q) {
                xj[q] = (double)((q < m ? fn - b.tau[m - 1 - q] : fn - (real)0.5) / fn);
                wj[q] = q < m ? (double)(b.omega[m - 1 - q] / fn) : 0.0;
            }
        }
    }
    return WQA_OK;
}

// Default rule of one direction on non-uniform knots: every row traced from its uniform
// rule (interior: the cardinal rule translated; boundary: the boundary rules, mirrored
// on the right), padded like the uniform rules.
wqa_status homotopy_direction(wqa_ctx *c, int kind, const LocalRule &interior, const std::vector<LocalRule> &boundary,
                              int dir, std::vector<double> &x, std::vector<double> &w) {
    const int p = c->p, Q = Q_of(c);
    const int64_t n = c->n[dir], nel = c->nel[dir];
    const real fn = (real)nel;
    const Knots kn = knots_of(c, dir);
    x.assign((size_t)n * Q, 0.0);
    w.assign((size_t)n * Q, 0.0);
    // rows are traced independently, on host threads (a trace costs milliseconds)
    std::vector<LocalRule> traced(n);
    std::vector<char> found(n, 0);
    for_rows(n, 4, [&](int64_t j0, int64_t j1) {
        for (int64_t j = j0; j < j1; ++j) {
            LocalRule uni;
            if (j >= p && j < n - p) {
                for (int q = 0; q < Q; ++q) {
                    uni.tau.push_back((real)(j - p) + interior.tau[q]);
                    uni.omega.push_back(interior.omega[q]);
                }
            } else if (j < p) {
                uni = boundary[j];
            } else {
                const LocalRule &b = boundary[n - 1 - j];
                const int m = (int)b.tau.size();
                for (int q = 0; q < m; ++q) {
                    uni.tau.push_back(fn - b.tau[m - 1 - q]);
                    uni.omega.push_back(b.omega[m - 1 - q]);
                }
            }
            found[j] = trace_row(p, kind, j, nel, c->brk[dir], uni, traced[j]);
        }
    });
    for (int64_t j = 0; j < n; ++j) {
        if (!found[j])
            return fail(WQA_ERULE, "%s rule of direction %d, row %lld: the homotopy from the uniform rule met a "
                        "singular point (no rule of this family on these knots)",
                        kind == WQA_MASS ? "mass" : "stiffness", dir, (long long)j);
        const LocalRule &r = traced[j];
        const real pad = j < p ? (kn.brk(0) + kn.brk(1)) / 2 : (kn.brk(nel - 1) + kn.brk(nel)) / 2;
        for (int q = 0; q < Q; ++q) {
            const bool real_node = q < (int)r.tau.size();
            x[j * Q + q] = (double)((real_node ? r.tau[q] : pad) / fn);
            w[j * Q + q] = real_node ? (double)(r.omega[q] / fn) : 0.0;
        }
    }
    return WQA_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------
extern "C" {

int wqa_abi_version(void) { return WQA_ABI_VERSION; }

const char *wqa_last_error(void) { return g_error.c_str(); }

wqa_status wqa_create(wqa_ctx **out, int hip_device) {
    if (!out) return fail(WQA_EINVAL, "wqa_create: out is NULL");
    *out = nullptr;
    if (hip_device < -1) return fail(WQA_EINVAL, "wqa_create: device %d", hip_device);
    if (hip_device >= 0) {
        int count = 0;
        hipError_t e = hipGetDeviceCount(&count);
        if (e != hipSuccess) return fail(WQA_EHIP, "hipGetDeviceCount: %s", hipGetErrorString(e));
        if (hip_device >= count) return fail(WQA_EINVAL, "wqa_create: device %d of %d", hip_device, count);
    }
    wqa_ctx *c = new (std::nothrow) wqa_ctx();
    if (!c) return fail(WQA_ENOMEM, "wqa_create: out of host memory");
    c->device = hip_device;
    *out = c;
    return ok();
}

void wqa_destroy(wqa_ctx *c) {
    if (!c) return;
    if (c->dev) {
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(c->dev);
    }
    delete c;
}

wqa_status wqa_set_space(wqa_ctx *c, int dim, int degree, const int64_t *n_elem) {
    if (!c || !n_elem) return fail(WQA_EINVAL, "wqa_set_space: NULL argument");
    if (dim != 2 && dim != 3) return fail(WQA_EUNSUPPORTED, "wqa_set_space: dim %d (supported: 2, 3)", dim);
    if (degree != 2 && degree != 3)
        return fail(WQA_EUNSUPPORTED, "wqa_set_space: degree %d (rules exist for 2 and 3)", degree);
    for (int k = 0; k < dim; ++k)
        if (n_elem[k] < degree + 1 || n_elem[k] > (int64_t)1 << 24)
            return fail(WQA_EINVAL, "wqa_set_space: n_elem[%d] = %lld (need degree+1 .. 2^24)", k,
                        (long long)n_elem[k]);
    int64_t rows = 1;
    for (int k = 0; k < dim; ++k) rows *= n_elem[k] + degree;
    if (rows > ((int64_t)1 << 40)) return fail(WQA_EINVAL, "wqa_set_space: %lld rows", (long long)rows);
    c->dim = dim;
    c->p = degree;
    c->pitch = 0;
    c->samples = WQA_SAMPLES_GRID;
    for (int k = 0; k < wqa::kMaxDim; ++k) {
        c->nel[k] = k < dim ? n_elem[k] : 0;
        c->n[k] = k < dim ? n_elem[k] + degree : 0;
        c->N[k] = c->n[k] * (degree + 1);
        c->brk[k].clear();
        for (int r = 0; r < 2; ++r) {
            c->have_rule[r][k] = false;
            c->nodes[r][k].clear();
            c->omega[r][k].clear();
            c->tab64[r][k].clear();
            c->tab32[r][k].clear();
        }
    }
    c->have_space = true;
    c->dev_current = false;
    return ok();
}

wqa_status wqa_set_knots(wqa_ctx *c, int dir, const double *breaks) {
    if (!c) return fail(WQA_EINVAL, "wqa_set_knots: NULL context");
    if (!c->have_space) return fail(WQA_ESTATE, "wqa_set_knots: call wqa_set_space first");
    if (dir < 0 || dir >= c->dim) return fail(WQA_EINVAL, "wqa_set_knots: dir %d of %d", dir, c->dim);
    const int64_t nel = c->nel[dir];
    std::vector<real> b;
    if (breaks) {
        if (breaks[0] != 0.0 || breaks[nel] != 1.0)
            return fail(WQA_EINVAL, "wqa_set_knots: breakpoints must run from 0 to 1 (got %g .. %g)", breaks[0],
                        breaks[nel]);
        for (int64_t e = 0; e < nel; ++e)
            if (!std::isfinite(breaks[e + 1]) || !(breaks[e + 1] - breaks[e] > 1e-12))
                return fail(WQA_EINVAL, "wqa_set_knots: breakpoints not strictly increasing at %lld", (long long)e);
        b.resize(nel + 1);
        for (int64_t e = 0; e <= nel; ++e) b[e] = (real)breaks[e] * (real)nel;
    }
    c->brk[dir] = b;
    for (int r = 0; r < 2; ++r) {
        c->have_rule[r][dir] = false;
        c->nodes[r][dir].clear();
        c->omega[r][dir].clear();
        c->tab64[r][dir].clear();
        c->tab32[r][dir].clear();
    }
    c->dev_current = false;
    return ok();
}

wqa_status wqa_set_default_rules(wqa_ctx *c) {
    if (!c) return fail(WQA_EINVAL, "wqa_set_default_rules: NULL context");
    if (!c->have_space) return fail(WQA_ESTATE, "wqa_set_default_rules: call wqa_set_space first");
    for (int kind = 0; kind < 2; ++kind) {
        LocalRule interior;
        if (!solve_interior(c->p, kind, interior))
            return fail(WQA_ERULE, "Newton found no admissible interior %s rule for p=%d",
                        kind ? "stiffness" : "mass", c->p);
        std::vector<LocalRule> boundary(c->p);
        for (int j = 0; j < c->p; ++j)
            if (!solve_boundary(c->p, kind, j, boundary[j]))
                return fail(WQA_ERULE, "Newton found no admissible boundary %s rule for p=%d row %d",
                            kind ? "stiffness" : "mass", c->p, j);
        for (int k = 0; k < c->dim; ++k) {
            std::vector<double> x, w;
            if (c->brk[k].empty()) {
                default_direction(c, interior, boundary, k, x, w);
            } else {
                wqa_status st = homotopy_direction(c, kind, interior, boundary, k, x, w);
                if (st != WQA_OK) return st;
            }
            // nodes travel as FP64 parameters in [0, 1]: each carries up to nel * 2^-53
            // element widths of rounding, which bounds the exactness any FP64 rule can show
            const double tol = std::max(1e-12, 8.0 * (double)c->nel[k] * 0x1p-53);
            wqa_status st = validate(c, kind, k, x.data(), w.data(), tol, c->brk[k].empty());
            if (st != WQA_OK) return st;
            st = install(c, kind, k, x.data(), w.data());
            if (st != WQA_OK) return st;
        }
    }
    return ok();
}

wqa_status wqa_set_rules(wqa_ctx *c, wqa_kind kind, int dir, int q, const double *nodes,
                         const double *weights, double exact_tol) {
    if (!c || !nodes || !weights) return fail(WQA_EINVAL, "wqa_set_rules: NULL argument");
    if (!c->have_space) return fail(WQA_ESTATE, "wqa_set_rules: call wqa_set_space first");
    if (kind != WQA_MASS && kind != WQA_STIFFNESS) return fail(WQA_EINVAL, "wqa_set_rules: kind %d", (int)kind);
    if (dir < 0 || dir >= c->dim) return fail(WQA_EINVAL, "wqa_set_rules: dir %d of %d", dir, c->dim);
    if (q != c->p + 1) return fail(WQA_EINVAL, "wqa_set_rules: q = %d, need degree + 1 = %d", q, c->p + 1);
    wqa_status st = validate(c, kind, dir, nodes, weights, exact_tol);
    if (st != WQA_OK) return st;
    st = install(c, kind, dir, nodes, weights);
    if (st != WQA_OK) return st;
    return ok();
}

wqa_status wqa_get_rules(const wqa_ctx *c, wqa_kind kind, int dir, double *nodes, double *weights) {
    if (!c) return fail(WQA_EINVAL, "wqa_get_rules: NULL context");
    if (kind != WQA_MASS && kind != WQA_STIFFNESS) return fail(WQA_EINVAL, "wqa_get_rules: kind %d", (int)kind);
    if (!c->have_space || dir < 0 || dir >= c->dim) return fail(WQA_EINVAL, "wqa_get_rules: dir %d", dir);
    if (!c->have_rule[kind][dir]) return fail(WQA_ESTATE, "wqa_get_rules: no rule installed");
    if (nodes) std::memcpy(nodes, c->nodes[kind][dir].data(), c->nodes[kind][dir].size() * 8);
    if (weights) std::memcpy(weights, c->omega[kind][dir].data(), c->omega[kind][dir].size() * 8);
    return ok();
}

wqa_status wqa_get_tables(const wqa_ctx *c, wqa_kind kind, int dir, double *out) {
    if (!c || !out) return fail(WQA_EINVAL, "wqa_get_tables: NULL argument");
    if (kind != WQA_MASS && kind != WQA_STIFFNESS) return fail(WQA_EINVAL, "wqa_get_tables: kind %d", (int)kind);
    if (!c->have_space || dir < 0 || dir >= c->dim) return fail(WQA_EINVAL, "wqa_get_tables: dir %d", dir);
    if (!c->have_rule[kind][dir]) return fail(WQA_ESTATE, "wqa_get_tables: no rule installed");
    std::memcpy(out, c->tab64[kind][dir].data(), c->tab64[kind][dir].size() * 8);
    return ok();
}

wqa_status wqa_query(const wqa_ctx *c, int64_t *n_rows, int64_t *slots_per_row,
                     int64_t *points_per_row, int64_t *grid_dims) {
    if (!c) return fail(WQA_EINVAL, "wqa_query: NULL context");
    if (!c->have_space) return fail(WQA_ESTATE, "wqa_query: no space set");
    int64_t rows = 1, slots = 1, pts = 1;
    for (int k = 0; k < c->dim; ++k) {
        rows *= c->n[k];
        slots *= S_of(c);
        pts *= Q_of(c);
    }
    if (n_rows) *n_rows = rows;
    if (slots_per_row) *slots_per_row = slots;
    if (points_per_row) *points_per_row = pts;
    if (grid_dims)
        for (int k = 0; k < c->dim; ++k) grid_dims[k] = c->N[k];
    return ok();
}

wqa_status wqa_set_final_mode(wqa_ctx *c, wqa_final mode) {
    if (!c) return fail(WQA_EINVAL, "wqa_set_final_mode: NULL context");
    if (mode != WQA_FINAL_PLAIN && mode != WQA_FINAL_DOT2 && mode != WQA_FINAL_F64)
        return fail(WQA_EINVAL, "wqa_set_final_mode: mode %d", (int)mode);
    c->final_mode = mode;
    return ok();
}

wqa_status wqa_set_grid_pitch(wqa_ctx *c, int64_t pitch) {
    if (!c) return fail(WQA_EINVAL, "wqa_set_grid_pitch: NULL context");
    if (!c->have_space) return fail(WQA_ESTATE, "wqa_set_grid_pitch: call wqa_set_space first");
    const int64_t Nd = c->N[c->dim - 1];
    if (pitch != 0 && (pitch < Nd || pitch % 4 != 0))
        return fail(WQA_EINVAL, "wqa_set_grid_pitch: pitch %lld (need 0, or a multiple of 4 of at least %lld)",
                    (long long)pitch, (long long)Nd);
    if (pitch != 0 && c->samples != WQA_SAMPLES_GRID)
        return fail(WQA_ESTATE, "wqa_set_grid_pitch: the pitch applies to the grid layout only (samples by row)");
    c->pitch = pitch;
    return ok();
}

wqa_status wqa_set_sample_layout(wqa_ctx *c, int layout) {
    if (!c) return fail(WQA_EINVAL, "wqa_set_sample_layout: NULL context");
    if (!c->have_space) return fail(WQA_ESTATE, "wqa_set_sample_layout: call wqa_set_space first");
    if (layout != WQA_SAMPLES_GRID && layout != WQA_SAMPLES_ROWS)
        return fail(WQA_EINVAL, "wqa_set_sample_layout: layout %d", layout);
    if (layout != WQA_SAMPLES_GRID && c->pitch != 0)
        return fail(WQA_ESTATE, "wqa_set_sample_layout: a grid pitch is set (reset it to 0 first)");
    c->samples = layout;
    return ok();
}

wqa_status wqa_set_dispatch_limit(wqa_ctx *c, int64_t max_tasks) {
    if (!c) return fail(WQA_EINVAL, "wqa_set_dispatch_limit: NULL context");
    if (max_tasks < 0) return fail(WQA_EINVAL, "wqa_set_dispatch_limit: %lld tasks", (long long)max_tasks);
    c->max_tasks = max_tasks == 0 ? wqa::kMaxTasksPerDispatch
                                  : std::min<int64_t>(max_tasks, wqa::kMaxTasksPerDispatch);
    return ok();
}

}  // extern "C"

namespace {

wqa_status ready(wqa_ctx *c, const char *who, wqa_dtype dtype) {
    if (!c) return fail(WQA_EINVAL, "%s: NULL context", who);
    if (c->device < 0) return fail(WQA_ESTATE, "%s: host-only context (created with device -1)", who);
    if (!c->have_space) return fail(WQA_ESTATE, "%s: call wqa_set_space first", who);
    if (!rules_complete(c)) return fail(WQA_ESTATE, "%s: rules missing (wqa_set_default_rules or wqa_set_rules)", who);
    if (dtype != WQA_F32 && dtype != WQA_F64) return fail(WQA_EINVAL, "%s: dtype %d", who, (int)dtype);
    wqa_status st = upload(c);
    if (st != WQA_OK) return st;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return fail(WQA_EHIP, "%s: hipSetDevice: %s", who, hipGetErrorString(e));
    return WQA_OK;
}

void fill(const wqa_ctx *c, wqa::DevSpace &sp, wqa::DevTabs &tb, wqa_dtype dtype) {
    sp.d = c->dim;
    sp.p = c->p;
    sp.ld = c->pitch ? c->pitch : c->N[c->dim - 1];
    sp.rows = c->samples == WQA_SAMPLES_ROWS ? 1 : 0;
    sp.band = 0;
    for (int k = 0; k < c->dim; ++k)
        if (c->banded[WQA_MASS][k] && c->banded[WQA_STIFFNESS][k]) sp.band |= 1 << k;
    for (int k = 0; k < wqa::kMaxDim; ++k) {
        sp.n[k] = c->n[k];
        sp.N[k] = c->N[k];
        for (int r = 0; r < 2; ++r) {
            tb.t[r][k] = dtype == WQA_F32 ? (const void *)c->d32[r][k] : (const void *)c->d64[r][k];
            tb.t64[r][k] = c->d64[r][k];
        }
    }
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

wqa_status forward(wqa_ctx *c, const char *who, wqa_dtype dtype, int what, const void *cf,
                   const void *const *a, void *M, void *K, void *stream) {
    wqa_status st = ready(c, who, dtype);
    if (st != WQA_OK) return st;
    if (!aligned16(cf) || !aligned16(M) || !aligned16(K))
        return fail(WQA_EINVAL, "%s: device buffers must be 16-byte aligned", who);
    if (a)
        for (int k = 0; k < c->dim; ++k)
            if (!aligned16(a[k])) return fail(WQA_EINVAL, "%s: a[%d] is not 16-byte aligned", who, k);
    if ((what & wqa::kWhatM) && (!cf || !M)) return fail(WQA_EINVAL, "%s: c and M must be non-NULL", who);
    if (what & wqa::kWhatK) {
        if (!a || !K) return fail(WQA_EINVAL, "%s: a and K must be non-NULL", who);
        for (int k = 0; k < c->dim; ++k)
            if (!a[k]) return fail(WQA_EINVAL, "%s: a[%d] is NULL", who, k);
    }
    wqa::DevSpace sp;
    wqa::DevTabs tb;
    fill(c, sp, tb, dtype);
    hipError_t e = wqa::launch_forward((int)dtype, c->final_mode, what, sp, tb, cf, a, M, K,
                                       (hipStream_t)stream, c->max_tasks);
    if (e != hipSuccess) return fail(WQA_EHIP, "%s: kernel launch: %s", who, hipGetErrorString(e));
    return ok();
}

wqa_status apply(wqa_ctx *c, const char *who, wqa_dtype dtype, int what, bool ones, const void *cf,
                 const void *const *a, const void *x, void *y, void *stream) {
    wqa_status st = ready(c, who, dtype);
    if (st != WQA_OK) return st;
    if (!y || (!ones && !x)) return fail(WQA_EINVAL, "%s: x and y must be non-NULL", who);
    if (!aligned16(x) || !aligned16(y) || !aligned16(cf))
        return fail(WQA_EINVAL, "%s: device buffers must be 16-byte aligned", who);
    if (what == wqa::kWhatM && !cf) return fail(WQA_EINVAL, "%s: the coefficient is NULL", who);
    if (what == wqa::kWhatK) {
        if (!a) return fail(WQA_EINVAL, "%s: a is NULL", who);
        for (int k = 0; k < c->dim; ++k) {
            if (!a[k]) return fail(WQA_EINVAL, "%s: a[%d] is NULL", who, k);
            if (!aligned16(a[k])) return fail(WQA_EINVAL, "%s: a[%d] is not 16-byte aligned", who, k);
        }
    }
    wqa::DevSpace sp;
    wqa::DevTabs tb;
    fill(c, sp, tb, dtype);
    // 3D products: the kernel blocked over all three directions; 2D products and the
    // load vector: the per-row kernel
    hipError_t e = (c->dim == 3 && !ones)
                       ? wqa::launch_apply_blocked((int)dtype, what, sp, tb, cf, a, x, y, (hipStream_t)stream,
                                                   c->max_tasks)
                       : wqa::launch_apply((int)dtype, what, ones, sp, tb, cf, a, x, y, (hipStream_t)stream,
                                           c->max_tasks);
    if (e != hipSuccess) return fail(WQA_EHIP, "%s: kernel launch: %s", who, hipGetErrorString(e));
    return ok();
}

}  // namespace

extern "C" {

wqa_status wqa_apply_mass(wqa_ctx *c, wqa_dtype dtype, const void *cf, const void *x, void *y, void *stream) {
    return apply(c, "wqa_apply_mass", dtype, wqa::kWhatM, false, cf, nullptr, x, y, stream);
}

wqa_status wqa_apply_stiffness(wqa_ctx *c, wqa_dtype dtype, const void *const *a, const void *x, void *y,
                               void *stream) {
    return apply(c, "wqa_apply_stiffness", dtype, wqa::kWhatK, false, nullptr, a, x, y, stream);
}

wqa_status wqa_assemble_load(wqa_ctx *c, wqa_dtype dtype, const void *f, void *b, void *stream) {
    return apply(c, "wqa_assemble_load", dtype, wqa::kWhatM, true, f, nullptr, nullptr, b, stream);
}

wqa_status wqa_assemble_mass(wqa_ctx *c, wqa_dtype dtype, const void *cf, void *M, void *stream) {
    return forward(c, "wqa_assemble_mass", dtype, wqa::kWhatM, cf, nullptr, M, nullptr, stream);
}

wqa_status wqa_assemble_stiffness(wqa_ctx *c, wqa_dtype dtype, const void *const *a, void *K,
                                  void *stream) {
    return forward(c, "wqa_assemble_stiffness", dtype, wqa::kWhatK, nullptr, a, nullptr, K, stream);
}

wqa_status wqa_assemble_fused(wqa_ctx *c, wqa_dtype dtype, const void *cf, const void *const *a,
                              void *M, void *K, void *stream) {
    return forward(c, "wqa_assemble_fused", dtype, wqa::kWhatMK, cf, a, M, K, stream);
}

wqa_status wqa_assemble_adjoint(wqa_ctx *c, wqa_dtype dtype, const void *gM, const void *gK,
                                void *dc, void *const *da, void *stream) {
    const char *who = "wqa_assemble_adjoint";
    wqa_status st = ready(c, who, dtype);
    if (st != WQA_OK) return st;
    if (!gM && !gK) return fail(WQA_EINVAL, "%s: gM and gK are both NULL", who);
    if ((gM == nullptr) != (dc == nullptr)) return fail(WQA_EINVAL, "%s: dc must be given exactly when gM is", who);
    if ((gK == nullptr) != (da == nullptr)) return fail(WQA_EINVAL, "%s: da must be given exactly when gK is", who);
    if (da)
        for (int k = 0; k < c->dim; ++k) {
            if (!da[k]) return fail(WQA_EINVAL, "%s: da[%d] is NULL", who, k);
            if (!aligned16(da[k])) return fail(WQA_EINVAL, "%s: da[%d] is not 16-byte aligned", who, k);
        }
    if (!aligned16(gM) || !aligned16(gK) || !aligned16(dc))
        return fail(WQA_EINVAL, "%s: device buffers must be 16-byte aligned", who);
    int what = (gM ? wqa::kWhatM : 0) | (gK ? wqa::kWhatK : 0);
    wqa::DevSpace sp;
    wqa::DevTabs tb;
    fill(c, sp, tb, dtype);
    hipError_t e = wqa::launch_adjoint((int)dtype, c->final_mode, what, sp, tb, gM, gK, dc, da,
                                       (hipStream_t)stream, c->max_tasks);
    if (e != hipSuccess) return fail(WQA_EHIP, "%s: kernel launch: %s", who, hipGetErrorString(e));
    return ok();
}

}  // extern "C"
