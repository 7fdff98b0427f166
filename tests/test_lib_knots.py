"""libwqa on non-uniform knots, host side (no kernel runs): the default rules traced by
the library's homotopy equal the oracle's (two independent solvers of the same
continuation), uniform breakpoints give back the uniform rules, bad breakpoints are
rejected and a path that meets a singular point is reported."""
import ctypes

import numpy as np
import pytest

from oracle import assembly as oa
from test_oracle_nonuniform import MESHES, N, perturbed


@pytest.fixture(scope="module")
def wqa():
    import paper_1710_01048_amd as mod
    return mod


@pytest.mark.parametrize("p", [2, 3])
def test_default_rules_match_oracle(wqa, p):
    breaks = [MESHES["graded"], MESHES["perturbed"]]
    sp = wqa.Space(2, p, (N, N), device=None, breaks=breaks)
    tabs = oa.rule_tables(p, (N, N), breaks)
    for k in range(2):
        for kind, kx, kw in ((wqa.MASS, "xM", "wM"), (wqa.STIFFNESS, "xK", "wK")):
            x, w = sp.rules(kind, k)
            assert np.abs(x.reshape(-1) - tabs[kx][k]).max() <= 1e-15
            assert np.abs(w.reshape(-1) - tabs[kw][k]).max() <= 1e-14 * np.abs(tabs[kw][k]).max()


@pytest.mark.parametrize("p", [2, 3])
def test_uniform_breakpoints_give_uniform_rules(wqa, p):
    n_el = (7, 5)
    a = wqa.Space(2, p, n_el, device=None)
    b = wqa.Space(2, p, n_el, device=None, breaks=[np.linspace(0, 1, 8), None])
    for kind in (wqa.MASS, wqa.STIFFNESS):
        xa, wa = a.rules(kind, 0)
        xb, wb = b.rules(kind, 0)
        assert np.abs(xa - xb).max() <= 1e-15 and np.abs(wa - wb).max() <= 1e-15
        assert np.array_equal(a.tables(kind, 1), b.tables(kind, 1))       # the uniform direction is untouched


def test_bad_breakpoints_rejected(wqa):
    with pytest.raises(wqa.WQAError, match="WQA_EINVAL"):
        wqa.Space(2, 2, (4, 4), device=None, breaks=[[0, 0.5, 0.4, 0.8, 1.0], None])
    with pytest.raises(wqa.WQAError, match="WQA_EINVAL"):
        wqa.Space(2, 2, (4, 4), device=None, breaks=[[0.1, 0.3, 0.5, 0.8, 1.0], None])
    with pytest.raises(ValueError):
        wqa.Space(2, 2, (4, 4), device=None, breaks=[[0, 0.5, 1.0], None])


def test_singular_path_reported(wqa):
    # the oracle's singular case: breakpoints moved by up to 0.3 element widths
    with pytest.raises(wqa.WQAError, match="WQA_ERULE.*singular point"):
        wqa.Space(2, 3, (N, N), device=None, breaks=[perturbed(N, amp=0.3), None])


def test_set_rules_validates_against_the_knots(wqa):
    # the uniform rule is not exact on graded knots: wqa_set_rules must refuse it there
    uni = wqa.Space(2, 3, (N, N), device=None)
    x, w = uni.rules(wqa.MASS, 0)
    sp = wqa.Space(2, 3, (N, N), device=None, rules=None, breaks=[MESHES["graded"], None])
    with pytest.raises(wqa.WQAError, match="WQA_ERULE"):
        sp.set_rules(wqa.MASS, 0, x, w)


@pytest.mark.parametrize("p", [2, 3])
def test_large_graded_mesh_every_row_exact(wqa, p):
    """160 elements graded as (k/N)^1.4: rows far from the origin move by ~10 element
    widths along the path.  Every traced rule is exact on the target knots, and the row
    whose trace once failed (130, stiffness) is the oracle's traced rule."""
    from oracle import nonuniform as nu
    n_el = 160
    breaks = [(k / n_el) ** 1.4 for k in range(n_el + 1)]
    sp = wqa.Space(2, p, (n_el, p + 1), device=None, breaks=[breaks, None])
    for kind, name in ((wqa.MASS, "mass"), (wqa.STIFFNESS, "stiffness")):
        x, w = sp.rules(kind, 0)
        worst = max(nu.exactness_residual(p, breaks, name, j, x[j], w[j]) for j in range(n_el + p))
        # FP64 nodes in [0, 1] carry ~n_el * 1e-16 element widths of rounding
        assert worst <= 1e-13, (name, worst)
    if p == 2:
        x, w = sp.rules(wqa.STIFFNESS, 0)
        tau, om = nu.row_rule(p, tuple(float(b) for b in breaks), "stiffness", 130)
        assert np.abs(x[130] * n_el - np.array([float(t) for t in tau])).max() <= 1e-12
        assert np.abs(w[130] * n_el - np.array([float(o) for o in om])).max() <= 1e-12
