"""Pins of the oracle's rules on non-uniform knots (homotopy continuation from the uniform
rules, oracle.nonuniform): uniform breakpoints give back the paper's rules; on graded and
randomly perturbed meshes every row is exact against Gram entries from scipy's B-splines
and Gauss-Legendre on the same knots; the continuation conditions hold; and the
constant-coefficient assembly equals the exact Galerkin matrices (Kronecker products)."""
import numpy as np
import pytest

import reference_1d as r1
import structured as st
from oracle import assembly as oa
from oracle import nonuniform as nu
from oracle import rules

N = 6


def graded(n):
    return tuple((k / n) ** 1.4 for k in range(n + 1))


def perturbed(n, seed=3, amp=0.15):
    # every interior breakpoint moved by up to amp element widths
    rng = np.random.default_rng(seed)
    b = np.arange(n + 1) / n + np.concatenate([[0], rng.uniform(-amp, amp, n - 1), [0]]) / n
    return tuple(float(x) for x in b)


MESHES = {"graded": graded(N), "perturbed": perturbed(N)}


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("kind", ["mass", "stiffness"])
def test_uniform_breaks_give_the_uniform_rules(p, kind):
    xs, ws = nu.direction_table(p, tuple(k / 5 for k in range(6)), kind)
    xu, wu = rules.direction_table(p, 5, kind)
    assert np.abs(np.array(xs) - np.array(xu)).max() <= 2e-16
    assert np.abs(np.array(ws) - np.array(wu)).max() <= 2e-16


@pytest.mark.parametrize("mesh", sorted(MESHES))
@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("kind", ["mass", "stiffness"])
def test_rows_exact_against_scipy_gram(mesh, p, kind):
    b = MESHES[mesh]
    xs, ws = nu.direction_table(p, b, kind)
    G = r1.gram(p, N, deriv=(kind == "stiffness"), breaks=b)
    n = N + p
    for j in range(n):
        x, w = np.array(xs[j]), np.array(ws[j])
        B = r1.basis_at(p, N, x, deriv=(kind == "stiffness"), breaks=b)        # [Q, n]
        quad = (w * B[:, j]) @ B                                                # row j against every column
        assert np.abs(quad - G[j]).max() <= 1e-13 * np.abs(G[j]).max(), (mesh, p, kind, j)


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("kind", ["mass", "stiffness"])
def test_continuation_conditions(p, kind):
    b = MESHES["graded"]
    xs, ws = nu.direction_table(p, b, kind)
    t = r1.knots(p, N, b)
    for j in range(p, N):                    # interior rows
        x, w = np.array(xs[j]), np.array(ws[j])
        elem = [(t[j + q], t[j + q + 1]) for q in range(p + 1)]
        rel = [(x[q] - a) / (c - a) for q, (a, c) in enumerate(elem)]
        assert all(0 < r < 1 for r in rel)                        # one node per element
        if kind == "mass" and p == 2:
            assert abs(rel[1] - 0.5) < 1e-14
        if p == 3:
            assert abs(rel[0] + rel[3] - 1) < 1e-14
        if kind == "stiffness" and p == 3:
            assert abs(w[0] * N - (t[j + 1] - t[j]) * N) < 1e-13    # omega_1 = first element length
        if kind == "stiffness" and p == 2:
            dB = r1.basis_at(p, N, x[1:2], deriv=True, breaks=b)[0, j]
            assert abs(dB) < 1e-12


@pytest.mark.parametrize("p,n_el,meshes", [(2, (6, 6), ("graded", "perturbed")),
                                           (3, (6, 5, 6), ("perturbed", None, "graded"))])
def test_constant_coefficients_equal_exact_galerkin(p, n_el, meshes):
    breaks = [None if m is None else MESHES[m] for m in meshes]
    if n_el[1] != N and meshes[1] is not None:
        raise AssertionError("mesh sizes")
    tabs = oa.rule_tables(p, n_el, breaks)
    d = len(n_el)
    shape = [(e + p) * (p + 1) for e in n_el]
    one = np.ones(shape)
    M, K = oa.assemble(p, n_el, tabs, c=one, a=[one] * d)
    Ms = [r1.gram(p, e, breaks=b) for e, b in zip(n_el, breaks)]
    Ks = [r1.gram(p, e, deriv=True, breaks=b) for e, b in zip(n_el, breaks)]
    M_ref = Ms[0]
    for X in Ms[1:]:
        M_ref = np.kron(M_ref, X)
    K_ref = 0
    for kk in range(d):
        Y = Ks[0] if kk == 0 else Ms[0]
        for k in range(1, d):
            Y = np.kron(Y, Ks[k] if k == kk else Ms[k])
        K_ref = K_ref + Y
    n = [e + p for e in n_el]
    assert np.abs(st.to_dense(M, n, p) - M_ref).max() <= 1e-14 * np.abs(M_ref).max()
    assert np.abs(st.to_dense(K, n, p) - K_ref).max() <= 1e-13 * np.abs(K_ref).max()


def test_singular_path_is_reported():
    # moving the breakpoints by up to 0.3 element widths drives the middle node of the
    # cubic stiffness rule of the third row from the right onto the zero of B'_j, where
    # its weight diverges: there is no such rule there, and the solver says so
    with pytest.raises(RuntimeError, match="homotopy lost the rule"):
        nu.row_rule(3, perturbed(N, amp=0.3), "stiffness", N + 3 - 3)
