"""Exact cost counts of the row rules, for the cost comparison of Sec. 3 (eq:Reduction
and the remark after it) and Sec. 4 (basis evaluations needed to build the mass matrix).

Two row rules on the uniform open knot vector of degree p:
  * "weighted_gauss": this method, p + 1 nodes per row and direction, one inside each
    element of supp(B_j) (Sec. 3);
  * "calabro": the row rules of Calabro et al. that the paper improves on, whose nodes
    are the knots and element midpoints inside supp(B_j): 2p + 1 per interior row.

Counts per interior row (a row whose support has p + 1 distinct elements):
  points      (p+1)^d          vs (2p+1)^d
  evaluations ((p+1)^2)^d      vs ((p+1)^2 + p^2)^d
The evaluation count of one direction is the number of nonzero basis functions at the
row's nodes: p + 1 at a point inside an element, p at an interior knot (one function
of the band vanishes there), so a knot node costs one evaluation less; evaluations of
functions that vanish are not counted (remark closing Sec. 4).  In d dimensions the
counts multiply over directions (eq:Decompo).

Unique points of a whole space: this method keeps its nodes per row, so rows never share
them (rows x (p+1)^d); the knot/midpoint nodes are shared between rows ((2 N_el + 1)^d
counting the boundary knots), which is the caveat of the remark after eq:Reduction.
"""
from fractions import Fraction
from math import prod


def points_per_row(p, d):
    return {"weighted_gauss": (p + 1) ** d, "calabro": (2 * p + 1) ** d}


def evaluations_per_row(p, d):
    return {"weighted_gauss": (p + 1) ** (2 * d), "calabro": ((p + 1) ** 2 + p ** 2) ** d}


def point_reduction(p, d):
    """((p+1)/(2p+1))^d (eq:Reduction)."""
    return Fraction(p + 1, 2 * p + 1) ** d


def evaluation_ratio(p, d):
    """Calabro evaluations over weighted-Gauss evaluations per interior row."""
    e = evaluations_per_row(p, d)
    return Fraction(e["calabro"], e["weighted_gauss"])


def unique_points(p, n_elem):
    n = [e + p for e in n_elem]
    return {"weighted_gauss": prod(n) * (p + 1) ** len(n), "calabro": prod(2 * e + 1 for e in n_elem)}


def report(p, n_elem):
    """Everything above for one space, JSON-friendly (ratios as floats)."""
    d = len(n_elem)
    return {"points_per_row": points_per_row(p, d),
            "evaluations_per_row": evaluations_per_row(p, d),
            "point_reduction": float(point_reduction(p, d)),
            "evaluation_ratio_calabro_over_ours": float(evaluation_ratio(p, d)),
            "unique_points": unique_points(p, n_elem)}
