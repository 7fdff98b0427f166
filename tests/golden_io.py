"""Readers for the paper fixtures under tests/golden (values quoted from the paper)."""
import os
from fractions import Fraction

import mpmath as mp

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line.split()


def number(text):
    """Exact Fraction for 'a/b' or integers, mpmath number for long decimals."""
    if "/" in text or text.lstrip("-").isdigit():
        return Fraction(text)
    return mp.mpf(text)


def interior_rules():
    """{(kind, p): {name: value}} from paper_interior_rules.txt."""
    out = {}
    for kind, p, name, value, *_ in _rows("paper_interior_rules.txt"):
        out.setdefault((kind, int(p)), {})[name] = number(value)
    return out


def wrong_cubic_root():
    return {name: mp.mpf(value) for name, value in _rows("paper_wrong_cubic_root.txt")}


def gram_rhs():
    """{(kind, p, offset): signed Fraction} from paper_gram_rhs.txt."""
    out = {}
    for kind, p, off, value, sign, *_ in _rows("paper_gram_rhs.txt"):
        v = Fraction(value)
        out[(kind, int(p), int(off))] = v if sign == "+" else -v
    return out


def count_ratios():
    return {int(p): (float(r), Fraction(inv)) for p, r, inv in _rows("paper_count_ratios.txt")}
