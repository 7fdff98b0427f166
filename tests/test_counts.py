"""Cost counts of the row rules (paper_1710_01048_amd.counts): the paper's quoted
reduction factors and evaluation ratios, and the per-row counts by brute force."""
import math
from fractions import Fraction
from itertools import product

import numpy as np
import pytest

import golden_io
from oracle import bspline as ob

PAPER = golden_io.count_ratios()


@pytest.fixture(scope="module")
def counts():
    from paper_1710_01048_amd import counts as mod
    return mod


@pytest.mark.parametrize("p", [2, 3])
def test_point_reduction_is_papers(counts, p):
    # eq:Reduction for d = 2, quoted as 25/9 and 49/16 in the remark closing Sec. 4
    assert 1 / counts.point_reduction(p, 2) == PAPER[p][1]


@pytest.mark.parametrize("p", [2, 3])
def test_evaluation_ratio_is_papers(counts, p):
    # the remark closing Sec. 4 prints 2.08 (p = 2) and 2.44 (p = 3); the exact ratios are
    # 169/81 = 2.0864 and 625/256 = 2.4414, which those figures truncate to two decimals
    r = counts.evaluation_ratio(p, 2)
    assert r == {2: Fraction(169, 81), 3: Fraction(625, 256)}[p]
    assert math.floor(100 * r) / 100 == PAPER[p][0]


def _nonzero(knots, p, n, x):
    return sum(1 for i in range(n) if ob.basis(knots, i, p, x) != 0)


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("d", [1, 2])
def test_counts_per_row_brute_force(counts, p, d):
    # count the basis functions that do not vanish at each node of an interior row,
    # exactly (Fractions), at the paper's interior nodes and at the knot/midpoint nodes
    import paper_1710_01048_amd as wqa
    n_el = 12
    knots = ob.open_uniform_knots(p, n_el, Fraction(1))
    n = n_el + p
    j = n // 2
    sp = wqa.Space(2, p, (n_el, n_el), device=None)
    x, w = sp.rules(wqa.MASS, 0)
    ours_1d = [Fraction(v).limit_denominator(10 ** 15) * n_el for v, wt in zip(x[j], w[j]) if wt != 0]
    lo, hi = knots[j], knots[j + p + 1]
    cal_1d = [lo + Fraction(k, 2) for k in range(1, 2 * int(hi - lo))]
    assert len(ours_1d) == p + 1 and len(cal_1d) == 2 * p + 1
    for nodes, key in ((ours_1d, "weighted_gauss"), (cal_1d, "calabro")):
        per_node = [_nonzero(knots, p, n, t) for t in nodes]
        # tensor product: B_a B_b is nonzero at (s, t) iff both factors are
        total = sum(np.prod([per_node[i] for i in idx]) for idx in product(range(len(nodes)), repeat=d))
        assert total == counts.evaluations_per_row(p, d)[key]
        assert len(nodes) ** d == counts.points_per_row(p, d)[key]


def test_unique_points(counts):
    u = counts.unique_points(3, (160, 160, 160))
    assert u["weighted_gauss"] == 163 ** 3 * 64 == 652 ** 3
    assert u["calabro"] == 321 ** 3
