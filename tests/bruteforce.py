"""Brute-force exact split search for tiny nodes (test helper).

Every candidate threshold is enumerated and scored with exact rational
arithmetic (``fractions.Fraction``) straight from the definition of Gini
impurity, Gini(S) = 1 - sum_c (s_c/|S|)^2, and of the decrease
G = Gini(P) - |L|/|P| Gini(L) - |R|/|P| Gini(R).  Nothing here shares code or
formulas with the oracle's exact-integer comparison.
"""
from __future__ import annotations

import math
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


def entropy(labels, n_classes) -> float:
    """H(S) = -sum_c p_c ln p_c with math.log (the library routine)."""
    n = len(labels)
    if n == 0:
        return 0.0
    h = 0.0
    for c in range(n_classes):
        k = sum(1 for y in labels if y == c)
        if k:
            h -= (k / n) * math.log(k / n)
    return h


def info_gain(left, right, n_classes) -> float:
    parent = list(left) + list(right)
    n = len(parent)
    return (entropy(parent, n_classes) - len(left) / n * entropy(left, n_classes)
            - len(right) / n * entropy(right, n_classes))


def all_bin_gains(bins_per_proj, labels, n_classes, n_bins):
    """[(gain, p, b, n_left)] of every histogram candidate with both sides non-empty."""
    out = []
    for p, bins in enumerate(bins_per_proj):
        for b in range(n_bins - 1):
            left = [y for k, y in zip(bins, labels) if k <= b]
            right = [y for k, y in zip(bins, labels) if k > b]
            if left and right:
                out.append((info_gain(left, right, n_classes), p, b, len(left)))
    return out


def all_threshold_gains(values_per_proj, labels, n_classes):
    """[(gain, p, t, n_left)] of every exact candidate (left = {v <= t})."""
    out = []
    for p, vals in enumerate(values_per_proj):
        for t in sorted(set(vals))[:-1]:
            left = [y for v, y in zip(vals, labels) if v <= t]
            right = [y for v, y in zip(vals, labels) if v > t]
            out.append((info_gain(left, right, n_classes), p, t, len(left)))
    return out
