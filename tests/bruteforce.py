"""Brute-force exact split search for tiny nodes (test helper).

Every candidate threshold is enumerated and scored with exact rational
arithmetic (``fractions.Fraction``) straight from the definition of Gini
impurity, Gini(S) = 1 - sum_c (s_c/|S|)^2, and of the decrease
G = Gini(P) - |L|/|P| Gini(L) - |R|/|P| Gini(R).  Nothing here shares code or
formulas with the oracle's exact-integer comparison.
"""
from __future__ import annotations

from fractions import Fraction


def gini(labels, n_classes) -> Fraction:
    n = len(labels)
    if n == 0:
        return Fraction(0)
    s = Fraction(0)
    for c in range(n_classes):
        p = Fraction(sum(1 for y in labels if y == c), n)
        s += p * p
    return 1 - s


def decrease(left, right, n_classes) -> Fraction:
    parent = list(left) + list(right)
    n = len(parent)
    return (gini(parent, n_classes)
            - Fraction(len(left), n) * gini(left, n_classes)
            - Fraction(len(right), n) * gini(right, n_classes))


def best_threshold_split(values_per_proj, labels, n_classes):
    """Exact split: every distinct value t (but the largest) of every projection,
    left = {v <= t}.  Ties go to the lowest projection, then the lowest t.
    Returns None when no split has a positive decrease, else (G, p, t, n_left)."""
    best = None
    for p, vals in enumerate(values_per_proj):
        for t in sorted(set(vals))[:-1]:
            left = [y for v, y in zip(vals, labels) if v <= t]
            right = [y for v, y in zip(vals, labels) if v > t]
            g = decrease(left, right, n_classes)
            if best is None or g > best[0]:
                best = (g, p, t, len(left))
    if best is None or best[0] <= 0:
        return None
    return best


def best_bin_split(bins_per_proj, labels, n_classes, n_bins):
    """Histogram split from given bin indices: boundaries b = 0..B-2, left =
    {bin <= b}.  Ties go to the lowest projection, then the lowest b."""
    best = None
    for p, bins in enumerate(bins_per_proj):
        for b in range(n_bins - 1):
            left = [y for k, y in zip(bins, labels) if k <= b]
            right = [y for k, y in zip(bins, labels) if k > b]
            if not left or not right:
                continue
            g = decrease(left, right, n_classes)
            if best is None or g > best[0]:
                best = (g, p, b, len(left))
    if best is None or best[0] <= 0:
        return None
    return best
