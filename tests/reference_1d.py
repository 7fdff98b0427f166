"""Independent 1D references built on scipy's B-spline evaluator and numpy's
Gauss-Legendre rule (library primitives, no code shared with the oracle or the
product): element-wise standard Gauss integration of basis products."""
import numpy as np
from scipy.interpolate import BSpline


def knots(p, n_el, breaks=None):
    b = np.linspace(0.0, 1.0, n_el + 1) if breaks is None else np.asarray(breaks, dtype=np.float64)
    return np.concatenate([np.zeros(p), b, np.ones(p)])


def basis_at(p, n_el, x, deriv=False, breaks=None):
    """[len(x), n] values of every basis function (or its derivative) at points x."""
    t = knots(p, n_el, breaks)
    n = n_el + p
    spl = BSpline(t, np.eye(n), p, extrapolate=False)
    if deriv:
        spl = spl.derivative()
    out = spl(np.asarray(x, dtype=np.float64))
    return np.nan_to_num(out)


def gauss_points(n_el, m, breaks=None):
    """All element-wise m-point Gauss-Legendre points and weights on [0, 1]."""
    g, w = np.polynomial.legendre.leggauss(m)
    b = np.linspace(0.0, 1.0, n_el + 1) if breaks is None else np.asarray(breaks, dtype=np.float64)
    h = np.diff(b)
    xs = b[:-1, None] + (g[None, :] + 1) / 2 * h[:, None]
    ws = w[None, :] * h[:, None] / 2
    return xs.reshape(-1), ws.reshape(-1)


def gram(p, n_el, deriv=False, m=None, coef=None, breaks=None):
    """Dense n x n matrix of int coef(x) phi_i phi_j over [0, 1] (phi = B or B')."""
    m = m or (p + 2)
    x, w = gauss_points(n_el, m, breaks)
    B = basis_at(p, n_el, x, deriv, breaks)
    ww = w if coef is None else w * coef(x)
    return (B * ww[:, None]).T @ B
