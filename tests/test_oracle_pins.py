"""Pins of the CPU oracle against things other than itself.

Each test checks the oracle against the mathematics or an independent routine:
brute-force enumeration with exact rationals, closed forms, a library
(scikit-learn's CART, numpy's float16 conversion), published test vectors, or
invariants that any correct split search satisfies.
"""
from __future__ import annotations

import bisect
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from tests import bruteforce as BF

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def one_node(X, y, C, feats, weights, *, T=0, bins=256, idx=None, hist=False, bin_mode=0, bin_seed=0,
             criterion=0):
    """Run the oracle on a single node holding all rows of X (or idx)."""
    n_rows = X.shape[1]
    idx = np.arange(n_rows, dtype=np.int32) if idx is None else np.asarray(idx, np.int32)
    k = len(feats)
    nz_off = np.zeros(k + 1, np.int32)
    nz_off[1:] = np.cumsum([len(f) for f in feats])
    nf = np.concatenate([np.asarray(f, np.int32) for f in feats])
    nw = np.concatenate([np.asarray(w, np.int8) for w in weights])
    sp, H = O.find_splits(X, y, C, np.array([0, len(idx)], np.int32), idx,
                          np.array([0, k], np.int32), nz_off, nf, nw, bins=bins,
                          sort_threshold=T, hist=hist, bin_mode=bin_mode, bin_seed=bin_seed,
                          criterion=criterion)
    return sp[0], H, (nz_off, nf, nw)


def exact_values(Xi, feats, weights, idx):
    """Projected values of integer-valued features, in exact integers."""
    return [[sum(int(w) * int(Xi[f, r]) for f, w in zip(fs, ws)) for r in idx]
            for fs, ws in zip(feats, weights)]


def random_projs(rng, k, d, zmax):
    feats, weights = [], []
    for _ in range(k):
        z = int(rng.integers(1, zmax + 1))
        feats.append(sorted(rng.choice(d, size=z, replace=False).tolist()))
        weights.append(rng.choice([-1, 1], size=z).tolist())
    return feats, weights


# --------------------------------------------------------------------------
# storage, projection, sampler
# --------------------------------------------------------------------------

def test_half_to_float_matches_numpy_on_every_pattern():
    bits = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)
    ref = bits.view(np.float16).astype(np.float32)
    got = np.array([O.half_to_float(int(b)) for b in bits], np.float32)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan].view(np.uint32), ref[~nan].view(np.uint32))


def test_projection_exact_on_integer_data():
    rng = np.random.default_rng(11)
    X = rng.integers(-1000, 1001, size=(12, 50)).astype(np.float32)
    for _ in range(200):
        z = int(rng.integers(1, 9))
        f = np.sort(rng.choice(12, size=z, replace=False)).astype(np.int32)
        w = rng.choice([-1, 1], size=z).astype(np.int8)
        r = int(rng.integers(0, 50))
        exact = sum(int(wj) * int(X[fj, r]) for fj, wj in zip(f, w))
        got = O.project_value(X, f, w, r)
        assert got == np.float32(exact)
        assert not (got == 0 and math.copysign(1.0, got) < 0), "projection produced -0.0"


def test_projection_error_within_z_ulp_of_fp64():
    rng = np.random.default_rng(12)
    X = (rng.standard_normal((16, 200)) * 10).astype(np.float32)
    for _ in range(300):
        z = int(rng.integers(1, 17))
        f = np.sort(rng.choice(16, size=z, replace=False)).astype(np.int32)
        w = rng.choice([-1, 1], size=z).astype(np.int8)
        r = int(rng.integers(0, 200))
        exact = sum(float(wj) * float(X[fj, r]) for fj, wj in zip(f, w))
        got = float(O.project_value(X, f, w, r))
        bound = z * max(abs(float(X[fj, r])) for fj in f) * 2.0 ** -23
        assert abs(got - exact) <= bound


def test_projection_sequential_csr_order():
    # a + b - c where the order matters in float32: 1e8 + 1 - 1e8 = 0 (not 1)
    X = np.array([[1e8], [1.0], [1e8]], np.float32)
    got = O.project_value(X, np.array([0, 1, 2], np.int32), np.array([1, 1, -1], np.int8), 0)
    assert got == np.float32(0.0)
    got2 = O.project_value(X, np.array([0, 2, 1], np.int32), np.array([1, -1, 1], np.int8), 0)
    assert got2 == np.float32(1.0)


def test_fp16_grid_projections_are_exact():
    # 1/256 grid, |x| <= 8: sums of <= 8 terms are exact in FP32 and FP16
    rng = np.random.default_rng(13)
    m = rng.integers(-2048, 2049, size=(10, 300))
    X32 = (m / 256.0).astype(np.float32)
    X16 = X32.astype(np.float16)
    assert np.array_equal(X16.astype(np.float32), X32)
    for _ in range(300):
        z = int(rng.integers(1, 9))
        f = np.sort(rng.choice(10, size=z, replace=False)).astype(np.int32)
        w = rng.choice([-1, 1], size=z).astype(np.int8)
        r = int(rng.integers(0, 300))
        exact = Fraction(sum(int(wj) * int(m[fj, r]) for fj, wj in zip(f, w)), 256)
        a, b = O.project_value(X32, f, w, r), O.project_value(X16, f, w, r)
        assert Fraction(float(a)) == exact and a == b


def test_splitmix64_published_vectors():
    with open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) as fh:
        rows = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    for c, val in rows:
        assert O.hash64(0, int(c)) == int(val, 16)


def test_sampler_counter_worked_by_hand():
    """The sampler's counter, c = ((((tree * 64 + level) * 2^24 + pos) * 2^10
    + proj) * 2^4 + draw), against integers worked out by hand: one field at
    a time (each lands at its own bit offset: draw 0, proj 4, pos 14, level
    38, tree 44), every field at its maximum (2^46 - 1), and a mixed case with
    a tree above 0 and the sign draw 15."""
    assert O.counter(0, 0, 0, 0, 15) == 15
    assert O.counter(0, 0, 0, 1, 0) == 16
    assert O.counter(0, 0, 1, 0, 0) == 16_384
    assert O.counter(0, 1, 0, 0, 0) == 274_877_906_944
    assert O.counter(1, 0, 0, 0, 0) == 17_592_186_044_416
    assert O.counter(3, 63, 16_777_215, 1023, 15) == 70_368_744_177_663
    # 133 * 2^38 = 36,558,761,623,552; 1000 * 2^14 = 16,384,000; 17 * 16 = 272
    assert O.counter(2, 5, 1000, 17, 15) == 36_558_778_007_839
    # a draw for tree 1 never collides with one of tree 0 at the largest level,
    # position, projection and draw
    assert O.counter(1, 0, 0, 0, 0) == O.counter(0, 63, 16_777_215, 1023, 15) + 1


def test_project_layout_against_a_plain_loop():
    """Blocks in node order, each [projection][sample] in frontier sample
    order, against a plain float32 loop over (node, projection, sample) on a
    frontier of uneven nodes (one empty) with uneven projection counts."""
    rng = np.random.default_rng(31)
    d, n_rows = 7, 50
    X = rng.standard_normal((d, n_rows)).astype(np.float32)
    sizes, ks = [5, 0, 3, 9], [2, 3, 1, 4]
    no = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    si = rng.integers(0, n_rows, size=int(no[-1])).astype(np.int32)
    po = np.concatenate([[0], np.cumsum(ks)]).astype(np.int32)
    feats, weights = random_projs(rng, int(po[-1]), d, 4)
    zo = np.concatenate([[0], np.cumsum([len(f) for f in feats])]).astype(np.int32)
    nf = np.concatenate([np.asarray(f, np.int32) for f in feats])
    nw = np.concatenate([np.asarray(w, np.int8) for w in weights])
    want = []
    for v in range(len(sizes)):
        for q in range(po[v], po[v + 1]):
            for i in range(no[v], no[v + 1]):
                acc = np.float32(0.0)
                for f, w in zip(feats[q], weights[q]):
                    acc = np.float32(acc + np.float32(w) * X[f, si[i]])
                want.append(acc)
    got = O.project(X, no, si, po, zo, nf, nw)
    assert got.shape == (sum(n * k for n, k in zip(sizes, ks)),)
    assert np.array_equal(got.view(np.uint32), np.array(want, np.float32).view(np.uint32))


def test_sampler_distinct_sorted_in_range_and_uniform():
    rng_counts = {}
    d, z = 5, 2
    for pos in range(20000):
        f, w = O.sample_projection(123, 0, 0, pos, 0, d, z)
        assert len(set(f.tolist())) == z and np.all(np.diff(f) > 0)
        assert f.min() >= 0 and f.max() < d
        assert set(w.tolist()) <= {-1, 1}
        rng_counts[tuple(f)] = rng_counts.get(tuple(f), 0) + 1
    # every one of the C(5,2) = 10 subsets equally likely: chi-square, 9 dof
    assert len(rng_counts) == 10
    exp = 20000 / 10
    chi2 = sum((v - exp) ** 2 / exp for v in rng_counts.values())
    assert chi2 < 27.9  # p = 0.001


def test_sampler_full_draw_and_determinism():
    f, _ = O.sample_projection(7, 3, 2, 11, 5, 12, 12)
    assert f.tolist() == list(range(12))
    a = O.sample_projection(99, 1, 4, 17, 3, 1024, 3)
    b = O.sample_projection(99, 1, 4, 17, 3, 1024, 3)
    assert a[0].tolist() == b[0].tolist() and a[1].tolist() == b[1].tolist()
    c = O.sample_projection(99, 2, 4, 17, 3, 1024, 3)
    assert c[0].tolist() != a[0].tolist() or c[1].tolist() != a[1].tolist()


def test_sampler_sign_balance():
    neg = tot = 0
    for pos in range(4000):
        _, w = O.sample_projection(5, 0, 1, pos, 7, 64, 3)
        neg += int((w < 0).sum())
        tot += w.size
    assert abs(neg / tot - 0.5) < 0.03


# --------------------------------------------------------------------------
# the density sampler (each feature kept with probability z/d) and FP32
# weights
# --------------------------------------------------------------------------

def _exact_binom_cdf(d, z, cap):
    """F(0), ..., F(cap-1) of Binomial(d, z/d) as exact rationals."""
    pi = Fraction(z, d)
    out, F = [], Fraction(0)
    for k in range(cap):
        F += math.comb(d, k) * pi**k * (1 - pi)**(d - k)
        out.append(F)
    return out


@pytest.mark.parametrize("d,z", [(64, 2), (1024, 2), (1024, 3), (10, 4), (20, 16), (300, 7)])
def test_density_count_is_the_exact_binomial_inversion(d, z):
    # The count is the least k with u < F(k), at most min(d, 16).  F is exact
    # here, so the oracle's binary64 recurrence may differ from it only where
    # u lies within a rounding margin of some F(k) (never, in practice).
    cap = min(d, 16)
    Fk = _exact_binom_cdf(d, z, cap)
    seed = 0xC0FFEE
    for pos in range(1500):
        h = O.hash64(seed ^ O.SEED_NNZ, O.counter(1, 2, pos, 3, 0))
        u = Fraction(h >> 11, 2**53)
        want = next((k for k in range(cap) if u < Fk[k]), cap)
        got = O.density_nnz(seed, 1, 2, pos, 3, d, z)
        if got != want:
            assert min(abs(u - F) for F in Fk) < Fraction(1, 2**40), (d, z, pos, got, want)


def test_density_count_law_is_binomial():
    from scipy import stats
    d, z, n = 48, 2, 20000
    got = np.array([O.density_nnz(11, 0, 0, pos, 0, d, z) for pos in range(n)])
    assert abs(got.mean() - z) < 0.05
    obs = np.bincount(got, minlength=17)[:17].astype(float)
    pmf = stats.binom.pmf(np.arange(17), d, z / d)
    pmf[16] += stats.binom.sf(16, d, z / d)
    exp = n * pmf
    keep = exp >= 5
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    chi2 = ((o - e) ** 2 / e).sum()
    assert stats.chi2.sf(chi2, len(o) - 1) > 1e-3


def test_density_count_cap_and_full_density():
    assert O.density_nnz(1, 0, 0, 0, 0, 5, 5) == 5        # z >= d: every feature
    assert O.density_nnz(1, 0, 0, 0, 0, 40, 40) == 16     # ... at most 16
    assert O.density_nnz(1, 0, 0, 0, 0, 3, 7) == 3
    got = [O.density_nnz(2, 0, 0, pos, 0, 20, 16) for pos in range(2000)]
    assert max(got) == 16 and min(got) >= 6               # Binomial(20, 0.8), capped


def test_density_projection_features_and_uniform_weights():
    from scipy import stats
    d = 30
    counts = np.zeros(d)
    ws, sizes = [], []
    for pos in range(6000):
        f, w = O.sample_projection(77, 0, 3, pos, 1, d, 2, O.SAMPLER_DENSITY, O.WEIGHTS_UNIFORM)
        assert f.size == w.size == O.density_nnz(77, 0, 3, pos, 1, d, 2)
        assert np.all(np.diff(f) > 0)
        if f.size:
            assert f.min() >= 0 and f.max() < d
        counts[f] += 1
        ws.append(w)
        sizes.append(f.size)
    assert 0 in sizes and max(sizes) >= 6
    # every feature equally likely (chi-square, d - 1 dof)
    assert stats.chisquare(counts).pvalue > 1e-3
    w = np.concatenate(ws).astype(np.float64)
    m = w * 2**24
    assert np.all(m == np.round(m)) and np.all(np.abs(m) % 2 == 1) and np.all(np.abs(w) < 1)
    assert stats.kstest(w, stats.uniform(loc=-1, scale=2).cdf).pvalue > 1e-3


def test_density_signs_are_balanced_and_fixed_law_keeps_its_stream():
    neg = tot = 0
    for pos in range(4000):
        _, w = O.sample_projection(5, 0, 1, pos, 7, 64, 3, O.SAMPLER_DENSITY, O.WEIGHTS_SIGN)
        assert set(w.tolist()) <= {-1.0, 1.0}
        neg += int((w < 0).sum())
        tot += w.size
    assert abs(neg / tot - 0.5) < 0.03
    # the fixed law with sign weights draws its signs from bit s of draw 15
    f, w = O.sample_projection(99, 1, 4, 17, 3, 1024, 3)
    bits = O.hash64(99, O.counter(1, 4, 17, 3, 15))
    assert [(-1.0 if (bits >> s) & 1 else 1.0) for s in range(3)] == w.tolist()


def test_projection_with_fp32_weights():
    from paper_2603_00326_amd import workloads as W
    rng = np.random.default_rng(8)
    X = rng.standard_normal((12, 500)).astype(np.float32)
    for _ in range(300):
        z = int(rng.integers(0, 9))
        f = np.sort(rng.choice(12, z, replace=False)).astype(np.int32)
        w = W.uniform_weights(rng, z)
        r = int(rng.integers(0, 500))
        v = O.project_value(X, f, w, r)
        if z == 0:
            assert v == 0
            continue
        # scaling by a power of two and negation commute with every rounding
        assert O.project_value(X, f, w * np.float32(4), r) == v * 4
        assert O.project_value(X, f, -w, r) == -v
        if z == 1:
            assert v == np.float32(w[0]) * X[f[0], r]
        # within the error bound of z products and z adds in FP32
        terms = [Fraction(float(w[j])) * Fraction(float(X[f[j], r])) for j in range(z)]
        bound = Fraction(2 * z, 2**24) * sum(abs(t) for t in terms)
        assert abs(Fraction(float(v)) - sum(terms)) <= bound


# --------------------------------------------------------------------------
# bins
# --------------------------------------------------------------------------

def test_bin_invariants_random():
    rng = np.random.default_rng(21)
    for _ in range(300):
        B = int(rng.integers(2, 257))
        v = (rng.standard_normal(64) * 10 ** rng.uniform(-3, 3)).astype(np.float32)
        lo, hi = v.min(), v.max()
        s = O.bin_scale(B, lo, hi)
        b = np.array([O.bin_index(x, lo, s, B) for x in np.sort(v)])
        assert b.min() >= 0 and b.max() <= B - 1
        assert np.all(np.diff(b) >= 0)          # monotone in v
        assert O.bin_index(lo, lo, s, B) == 0
        assert O.bin_index(hi, lo, s, B) == B - 1


def test_bins_equal_exact_floor_away_from_rounding():
    rng = np.random.default_rng(22)
    checked = 0
    for _ in range(200):
        B = int(rng.choice([2, 3, 7, 16, 100, 128, 255, 256]))
        v = rng.integers(-500, 501, size=40).astype(np.float32)
        lo, hi = v.min(), v.max()
        if lo == hi:
            continue
        s = O.bin_scale(B, lo, hi)
        for x in v:
            e = Fraction(int(x) - int(lo)) * B / (int(hi) - int(lo))
            if e >= B:
                assert O.bin_index(x, lo, s, B) == B - 1
                continue
            if abs(e - round(e)) < Fraction(1, 10**5) * max(1, e):
                continue        # too close to a boundary for the rounding to be decided
            assert O.bin_index(x, lo, s, B) == math.floor(e)
            checked += 1
    assert checked > 1000


def test_scale_overflow_guard():
    lo = np.float32(1.0)
    hi = np.nextafter(lo, np.float32(2.0))
    # hi - lo = 2^-23: 256 / 2^-23 = 2^31, finite; a denormal width overflows
    assert O.bin_scale(256, lo, hi) == np.float32(2.0 ** 31)
    tiny = np.float32(1e-45)
    assert O.bin_scale(256, np.float32(0), tiny) == np.finfo(np.float32).max
    assert O.bin_scale(256, np.float32(3), np.float32(3)) == np.finfo(np.float32).max
    assert O.bin_index(np.float32(3), np.float32(3), np.finfo(np.float32).max, 256) == 0


def test_worked_example():
    spec = {}
    with open(os.path.join(GOLDEN, "worked_separable.txt")) as fh:
        for ln in fh:
            if ln.strip() and not ln.startswith("#"):
                key, *vals = ln.split()
                spec[key] = vals
    v = np.array([float(t) for t in spec["values"]], np.float32)
    y = np.array([int(t) for t in spec["labels"]], np.int32)
    B = int(spec["bins"][0])
    s = O.bin_scale(B, v.min(), v.max())
    assert [O.bin_index(x, v.min(), s, B) for x in v] == [int(t) for t in spec["expect_bins"]]
    sp, H, _ = one_node(v[None, :], y, 2, [[0]], [[1]], bins=B, hist=True)
    assert sp["proj"] == 0 and sp["kind"] == 0
    assert sp["bin"] == int(spec["expect_split_bin"][0])
    assert sp["n_left"] == int(spec["expect_n_left"][0])
    assert sp["gain"] == float(Fraction(int(spec["expect_gain_num"][0]), int(spec["expect_gain_den"][0])))
    assert H[0].sum() == 4 and H[0, :, 0].sum() == 2


# --------------------------------------------------------------------------
# split search: brute force, closed forms, library, invariants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(60))
def test_sort_path_matches_bruteforce(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(2, 13))
    C = int(rng.integers(2, 5))
    d = 6
    Xi = rng.integers(-3, 4, size=(d, n))
    y = rng.integers(0, C, size=n).astype(np.int32)
    k = int(rng.integers(1, 5))
    feats, weights = random_projs(rng, k, d, 3)
    vals = exact_values(Xi, feats, weights, range(n))
    want = BF.best_threshold_split(vals, y.tolist(), C)
    sp, _, _ = one_node(Xi.astype(np.float32), y, C, feats, weights, T=1 << 30)
    assert sp["kind"] == 1
    if want is None:
        assert sp["proj"] == -1 and sp["gain"] == 0.0 and sp["n_left"] == n
        return
    g, p, t, n_left = want
    assert sp["proj"] == p and sp["threshold"] == np.float32(t) and sp["n_left"] == n_left
    assert sp["bin"] == n_left - 1 and sp["n_right"] == n - n_left
    assert abs(Fraction(float(sp["gain"])) - g) <= g * Fraction(1, 2**50)


@pytest.mark.parametrize("seed", range(120))
def test_hist_path_matches_bruteforce(seed):
    rng = np.random.default_rng(2000 + seed)
    n = int(rng.integers(2, 13))
    C = int(rng.integers(2, 5))
    d = 5
    amp = int(rng.choice([4, 1000]))
    Xi = rng.integers(-amp, amp + 1, size=(d, n))
    y = rng.integers(0, C, size=n).astype(np.int32)
    k = int(rng.integers(1, 5))
    B = int(rng.choice([2, 3, 4, 7, 8, 16, 100, 256]))
    feats, weights = random_projs(rng, k, d, 3)
    vals = exact_values(Xi, feats, weights, range(n))
    bins = []
    for vs in vals:
        lo, hi = min(vs), max(vs)
        row = []
        # B/(hi-lo) exactly representable in binary32: then (v-lo)*scale is the
        # exact rational e whenever e is an integer, and no edge is ambiguous
        exact_scale = hi != lo and Fraction(float(np.float32(B) / np.float32(hi - lo))) == Fraction(B, hi - lo)
        for v in vs:
            if hi == lo:
                row.append(0)
                continue
            e = Fraction(v - lo) * B / (hi - lo)
            near = abs(e - round(e)) < Fraction(1, 10**5) * max(1, e)
            if e < B and e != 0 and near and not (exact_scale and e.denominator == 1):
                pytest.skip("a sample sits on a bin edge within rounding")
            row.append(min(math.floor(e), B - 1))
        bins.append(row)
    want = BF.best_bin_split(bins, y.tolist(), C, B)
    sp, H, _ = one_node(Xi.astype(np.float32), y, C, feats, weights, T=0, bins=B, hist=True)
    assert sp["kind"] == 0
    for p in range(k):
        for b in range(B):
            for c in range(C):
                assert H[p, b, c] == sum(1 for kk, yy in zip(bins[p], y) if kk == b and yy == c)
    if want is None:
        assert sp["proj"] == -1 and sp["gain"] == 0.0
        return
    g, p, b, n_left = want
    assert (sp["proj"], sp["bin"], sp["n_left"]) == (p, b, n_left)
    assert abs(Fraction(float(sp["gain"])) - g) <= g * Fraction(1, 2**50)


@pytest.mark.parametrize("seed", range(25))
def test_hist_equals_sort_when_bins_hold_single_values(seed):
    # small-integer projected values and B >= range + 1: each nonempty bin holds
    # one distinct value, so both paths must pick the same partition
    rng = np.random.default_rng(3000 + seed)
    n = int(rng.integers(4, 200))
    C = int(rng.integers(2, 5))
    d = 8
    X = rng.integers(0, 3, size=(d, n)).astype(np.float32)
    y = rng.integers(0, C, size=n).astype(np.int32)
    feats, weights = random_projs(rng, 6, d, 3)
    sh, _, csr = one_node(X, y, C, feats, weights, T=0, bins=256)
    ss, _, _ = one_node(X, y, C, feats, weights, T=1 << 30, bins=256)
    assert sh["proj"] == ss["proj"]
    assert sh["n_left"] == ss["n_left"] and sh["gain"] == ss["gain"]
    if sh["proj"] >= 0:
        no, si, po = np.array([0, n], np.int32), np.arange(n, dtype=np.int32), np.array([0, 6], np.int32)
        a, _ = O.partition(X, no, si, po, *csr, sh[None], bins=256)
        b, _ = O.partition(X, no, si, po, *csr, ss[None], bins=256)
        assert np.array_equal(a, b)


def test_closed_forms():
    X = np.array([[0.0, 1.0, 2.0, 3.0]], np.float32)
    y = np.array([0, 0, 1, 1], np.int32)
    for T in (0, 1 << 30):
        sp, _, _ = one_node(X, y, 2, [[0]], [[1]], T=T)
        assert sp["gain"] == 0.5 and sp["n_left"] == 2          # separable: G = Gini(parent)
    # three pure classes of sizes 2, 3, 5 separated by one threshold at best:
    X3 = np.array([[0, 0, 1, 1, 1, 2, 2, 2, 2, 2]], np.float32)
    y3 = np.array([0, 0, 1, 1, 1, 2, 2, 2, 2, 2], np.int32)
    sp, _, _ = one_node(X3, y3, 3, [[0]], [[1]], T=1 << 30)
    parent = 1 - Fraction(4 + 9 + 25, 100)
    # split {0,1} | {2}: left Gini = 1 - (4+9)/25 = 12/25 with weight 1/2
    g = parent - Fraction(1, 2) * Fraction(12, 25)
    assert abs(Fraction(float(sp["gain"])) - g) < Fraction(1, 2**50)
    # constant projection: no candidate
    sp, _, _ = one_node(np.ones((1, 6), np.float32), np.array([0, 1] * 3, np.int32), 2, [[0]], [[1]])
    assert sp["proj"] == -1 and sp["gain"] == 0.0
    # pure node: no split
    sp, _, _ = one_node(np.arange(6, dtype=np.float32)[None], np.zeros(6, np.int32), 2, [[0]], [[1]])
    assert sp["proj"] == -1 and sp["n_left"] == 6


def test_tie_rules():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((4, 64)).astype(np.float32)
    y = (X[1] > 0).astype(np.int32)
    for T in (0, 1 << 30):
        # the same projection at indices 0 and 1: the lower index wins
        sp, _, _ = one_node(X, y, 2, [[1, 2], [1, 2]], [[1, -1], [1, -1]], T=T)
        assert sp["proj"] == 0
        # w and -w give mirrored splits with equal Gini: the lower index wins
        sp, _, _ = one_node(X, y, 2, [[1], [1]], [[1], [-1]], T=T)
        assert sp["proj"] == 0
        sp, _, _ = one_node(X, y, 2, [[3], [1], [1]], [[1], [-1], [1]], T=T)
        assert sp["proj"] == 1
    # empty bins: the chosen bin is the last nonempty one on the left
    Xe = np.array([[0.0, 0.0, 10.0, 10.0]], np.float32)
    ye = np.array([0, 0, 1, 1], np.int32)
    sp, H, _ = one_node(Xe, ye, 2, [[0]], [[1]], bins=256, hist=True)
    assert sp["bin"] == 0 and H[0, 0].sum() == 2 and H[0, 255].sum() == 2
    # symmetric counts (3,1 | 1,3) vs (1,3 | 3,1): equal Q, the lower index wins
    Xs = np.array([[0, 0, 0, 1, 1, 1, 1, 0], [1, 1, 1, 0, 0, 0, 0, 1]], np.float32)
    ys = np.array([0, 0, 0, 1, 1, 1, 0, 1], np.int32)
    sp, _, _ = one_node(Xs, ys, 2, [[0], [1]], [[1], [1]], T=1 << 30)
    assert sp["proj"] == 0


def test_gain_matches_sklearn_cart():
    sk = pytest.importorskip("sklearn.tree")
    rng = np.random.default_rng(31)
    for trial in range(20):
        n = int(rng.integers(20, 400))
        C = int(rng.integers(2, 5))
        X = rng.standard_normal((3, n)).astype(np.float32)
        y = rng.integers(0, C, size=n).astype(np.int32)
        feats, weights = [[0, 2]], [[1, -1]]
        sp, _, _ = one_node(X, y, C, feats, weights, T=1 << 30)
        v = np.array([O.project_value(X, np.array([0, 2], np.int32), np.array([1, -1], np.int8), r)
                      for r in range(n)], np.float32)
        t = sk.DecisionTreeClassifier(max_depth=1, criterion="gini", random_state=0).fit(v[:, None], y)
        if t.tree_.node_count == 1:
            assert sp["proj"] == -1
            continue
        imp, cnt = t.tree_.impurity, t.tree_.n_node_samples
        dec = imp[0] - cnt[1] / cnt[0] * imp[1] - cnt[2] / cnt[0] * imp[2]
        assert sp["proj"] == 0
        assert abs(sp["gain"] - dec) <= 1e-9 * max(dec, 1e-12)


@pytest.mark.parametrize("seed", range(10))
def test_invariants_random_frontier(seed):
    from paper_2603_00326_amd import workloads as W
    rng = np.random.default_rng(seed)
    sizes = rng.integers(0, 300, size=12)
    C = int(rng.integers(2, 8))
    wl = W.random_frontier(4000 + seed, n_rows=2000, d=20, n_classes=C, sizes=sizes, k=8, z=3,
                           bins=int(rng.choice([16, 128, 256])), sort_threshold=int(rng.integers(0, 200)))
    sp, H = O.find_splits_w(wl, hist=True)
    for v in range(wl.n_nodes):
        a, b = wl.node_offsets[v], wl.node_offsets[v + 1]
        yy = wl.y[wl.sample_idx[a:b]]
        n = b - a
        assert sp[v]["n_left"] + sp[v]["n_right"] == n
        parent = [int((yy == c).sum()) for c in range(C)]
        g_parent = 1 - sum(Fraction(p, n) ** 2 for p in parent) if n else 0
        if sp[v]["proj"] >= 0:
            assert 0 < sp[v]["gain"] <= float(g_parent) * (1 + 1e-12)
            assert sp[v]["n_left"] >= 1 and sp[v]["n_right"] >= 1
        else:
            assert sp[v]["gain"] == 0
        hist_node = n >= wl.sort_threshold
        assert sp[v]["kind"] == (0 if hist_node else 1)
        for q in range(wl.proj_offsets[v], wl.proj_offsets[v + 1]):
            if hist_node:
                assert H[q].sum() == n
                assert H[q].sum(axis=0).tolist() == parent
            else:
                assert H[q].sum() == 0
    # partition: a stable permutation with the split's left count
    out, co = O.partition(wl.X, wl.node_offsets, wl.sample_idx, wl.proj_offsets, wl.nz_offsets,
                          wl.nz_feature, wl.nz_weight, sp, bins=wl.bins)
    for v in range(wl.n_nodes):
        a, b = wl.node_offsets[v], wl.node_offsets[v + 1]
        assert co[2 * v] == a and co[2 * v + 1] - a == sp[v]["n_left"]
        assert sorted(out[a:b].tolist()) == sorted(wl.sample_idx[a:b].tolist())
        src = wl.sample_idx[a:b].tolist()
        left, right = out[a:co[2 * v + 1]].tolist(), out[co[2 * v + 1]:b].tolist()
        pos = {}
        for i, r in enumerate(src):
            pos.setdefault(r, []).append(i)
        # order preserved within each child (positions in the input increase)
        for part in (left, right):
            seen = {}
            last = -1
            for r in part:
                i = pos[r][seen.get(r, 0)]
                seen[r] = seen.get(r, 0) + 1
                assert i > last
                last = i
    assert co[-1] == wl.node_offsets[-1]


def test_partition_matches_list_comprehension_on_integer_data():
    rng = np.random.default_rng(41)
    d, n = 6, 300
    Xi = rng.integers(-5, 6, size=(d, n))
    X = Xi.astype(np.float32)
    y = rng.integers(0, 3, size=n).astype(np.int32)
    idx = rng.permutation(n)[:200].astype(np.int32)
    feats, weights = random_projs(rng, 5, d, 3)
    for T in (0, 1 << 30):
        sp, _, csr = one_node(X, y, 3, feats, weights, T=T, idx=idx)
        if sp["proj"] < 0:
            continue
        vals = exact_values(Xi, [feats[sp["proj"]]], [weights[sp["proj"]]], idx)[0]
        if T:
            goes = [v <= float(sp["threshold"]) for v in vals]
        else:
            lo, hi = min(vals), max(vals)
            goes = [min(math.floor(Fraction(v - lo) * 256 / (hi - lo)), 255) <= sp["bin"] for v in vals]
        want = [r for r, g in zip(idx, goes) if g] + [r for r, g in zip(idx, goes) if not g]
        got, co = O.partition(X, np.array([0, len(idx)], np.int32), idx, np.array([0, 5], np.int32),
                              *csr, sp[None], bins=256)
        assert got.tolist() == [int(r) for r in want] and co[1] == sum(goes)


def test_fp16_storage_equals_fp32_storage():
    from paper_2603_00326_amd import workloads as W
    X32 = W.grid_matrix(3, 5000, 16)
    rng = np.random.default_rng(3)
    y = rng.integers(0, 2, size=5000).astype(np.int32)
    po, no, nf, nw = W.random_projections(rng, 1, 24, 16, (1, 8))
    args = (np.array([0, 5000], np.int32), np.arange(5000, dtype=np.int32), po, no, nf, nw)
    a, Ha = O.find_splits(X32, y, 2, *args, hist=True)
    b, Hb = O.find_splits(X32.astype(np.float16), y, 2, *args, hist=True)
    assert a.tobytes() == b.tobytes() and np.array_equal(Ha, Hb)


# --------------------------------------------------------------------------
# growth
# --------------------------------------------------------------------------

def _route(nodes, X, r, root):
    i = root
    while not nodes[i]["is_leaf"]:
        nd = nodes[i]
        z = nd["nnz"]
        v = O.project_value(X, nd["feature"][:z], nd["weight"][:z], r)
        if nd["kind"] == 0:
            left = O.bin_index(v, nd["lo"], nd["scale"], nd["n_bins"]) <= nd["bin"]
        else:
            left = v <= nd["threshold"]
        i = nd["left"] if left else nd["right"]
    return i


SAMPLERS = [(O.SAMPLER_FIXED, O.WEIGHTS_SIGN), (O.SAMPLER_DENSITY, O.WEIGHTS_UNIFORM),
            (O.SAMPLER_DENSITY, O.WEIGHTS_SIGN)]


# (criterion, bin layout) of growth: Gini or entropy, equal- or random-width bins
GROW_MODES = [(O.CRIT_GINI, O.BINS_EQUAL), (O.CRIT_ENTROPY, O.BINS_EQUAL), (O.CRIT_GINI, O.BINS_RANDOM),
              (O.CRIT_ENTROPY, O.BINS_RANDOM)]
GROW_CASES = [(s, w, O.CRIT_GINI, O.BINS_EQUAL) for s, w in SAMPLERS] + \
             [(O.SAMPLER_FIXED, O.WEIGHTS_SIGN, c, b) for c, b in GROW_MODES[1:]] + \
             [(O.SAMPLER_DENSITY, O.WEIGHTS_UNIFORM, O.CRIT_ENTROPY, O.BINS_RANDOM)]


@pytest.mark.parametrize("sampler,weights,criterion,bin_mode", GROW_CASES)
def test_growth_to_purity_small(sampler, weights, criterion, bin_mode):
    rng = np.random.default_rng(51)
    d, n, C = 10, 400, 3
    X = rng.standard_normal((d, n)).astype(np.float32)
    y = rng.integers(0, C, size=n).astype(np.int32)
    roots = [np.sort(np.random.default_rng(t).integers(0, n, n)).astype(np.int32) for t in range(3)]
    ro = np.array([0, n, 2 * n, 3 * n], np.int64)
    ri = np.concatenate(roots)
    nodes, ln, lu = O.grow_forest(X, y, C, ro, ri, k=6, z=2, seed=9, bins=64, sort_threshold=50,
                                  sampler=sampler, weights=weights, criterion=criterion, bin_mode=bin_mode,
                                  bin_seed=31)
    assert ln[0] == 3
    # the split kinds follow the switch and the bin layout: sort below 50
    # samples, random-width (kind 2) or equal-width (kind 0) histograms above
    internal_ = nodes[nodes["is_leaf"] == 0]
    hist_kind = 2 if bin_mode == O.BINS_RANDOM else 0
    assert np.all(internal_["kind"] == np.where(internal_["n_samples"] < 50, 1, hist_kind))
    for t in range(3):
        for r in roots[t]:
            leaf = _route(nodes, X, int(r), t)
            assert nodes[leaf]["tree"] == t
    leaves = nodes[nodes["is_leaf"] == 1]
    internal = nodes[nodes["is_leaf"] == 0]
    assert np.all(internal["gain"] > 0)
    # an internal node's projection has 1..16 distinct ascending features and
    # nonzero weights of its law; nothing past nnz
    for nd in internal:
        z = int(nd["nnz"])
        assert 1 <= z <= 16 and np.all(np.diff(nd["feature"][:z]) > 0)
        w = nd["weight"][:z].astype(np.float64)
        if weights == O.WEIGHTS_SIGN:
            assert set(w.tolist()) <= {-1.0, 1.0}
        else:
            assert np.all((np.abs(w) < 1) & (w != 0))
        assert not nd["feature"][z:].any() and not nd["weight"][z:].any()
    if sampler == O.SAMPLER_DENSITY:
        assert len(set(internal["nnz"].tolist())) > 1
    # every sample of each tree lands in exactly one leaf: leaf sizes sum to n
    for t in range(3):
        assert leaves[leaves["tree"] == t]["n_samples"].sum() == n
    # children sizes add up
    for nd in internal:
        assert nodes[nd["left"]]["n_samples"] + nodes[nd["right"]]["n_samples"] == nd["n_samples"]
    # training accuracy on the bootstrap rows is 100% (continuous features: no
    # duplicate rows with different labels)
    acc = np.mean([nodes[_route(nodes, X, int(r), t)]["label"] == y[r]
                   for t in range(3) for r in roots[t]])
    assert acc == 1.0


def renumber_tree(nodes, t):
    """Nodes of tree t with ids rewritten to the tree's own creation order."""
    sel = np.nonzero(nodes["tree"] == t)[0]
    remap = {int(g): i for i, g in enumerate(sel)}
    out = nodes[sel].copy()
    for f in ("parent", "left", "right"):
        out[f] = [remap.get(int(g), -1) if g >= 0 else -1 for g in out[f]]
    return out


@pytest.mark.parametrize("sampler,weights,criterion,bin_mode", GROW_CASES)
def test_growth_batched_equals_single_tree(sampler, weights, criterion, bin_mode):
    # Random-width bins of growth are keyed by tree position, so a node's bins
    # (and hence every tree) do not depend on the other trees of the batch; a
    # key taken from the node's place in the batched frontier would fail this.
    rng = np.random.default_rng(52)
    d, n, C = 8, 300, 2
    X = rng.standard_normal((d, n)).astype(np.float32)
    y = rng.integers(0, C, size=n).astype(np.int32)
    roots = [np.sort(np.random.default_rng(100 + t).integers(0, n, n)).astype(np.int32) for t in range(3)]
    ro = np.array([0, n, 2 * n, 3 * n], np.int64)
    kw = dict(sampler=sampler, weights=weights, criterion=criterion, bin_mode=bin_mode, bin_seed=5)
    nodes, _, _ = O.grow_forest(X, y, C, ro, np.concatenate(roots), k=5, z=2, seed=4, bins=32,
                                sort_threshold=20, **kw)
    for t in range(3):
        single, _, _ = O.grow_forest(X, y, C, np.array([0, n], np.int64), roots[t], k=5, z=2, seed=4,
                                     bins=32, sort_threshold=20, first_tree=t, **kw)
        assert renumber_tree(nodes, t).tobytes() == single.tobytes()


def test_growth_random_width_key_is_the_tree_position():
    """The random-width bins of a grown node come from the width stream keyed
    by (tree, level, pos, p): rebuilding the root's split from its recorded
    projection, the keyed boundaries over the root's [lo, hi] and the
    oracle's one-level search at that key reproduces the recorded threshold."""
    rng = np.random.default_rng(53)
    d, n, C = 6, 500, 2
    X = rng.standard_normal((d, n)).astype(np.float32)
    y = (X[0] + X[1] > 0).astype(np.int32)
    ri = np.arange(n, dtype=np.int32)
    tree = 7
    nodes, _, _ = O.grow_forest(X, y, C, np.array([0, n], np.int64), ri, k=4, z=2, seed=3, bins=16,
                                max_depth=1, first_tree=tree, bin_mode=O.BINS_RANDOM, bin_seed=99)
    root = nodes[0]
    assert root["is_leaf"] == 0 and root["kind"] == 2
    z = int(root["nnz"])
    v = np.array([O.project_value(X, root["feature"][:z], root["weight"][:z], r) for r in range(n)], np.float32)
    lo, hi = v.min(), v.max()
    assert np.float32(root["lo"]) == lo
    # which of the node's 4 projections won is not recorded; one of the keys
    # (tree, level 0, pos 0, p) must give boundaries containing the threshold
    # at the recorded bin, and routing by it must give the recorded children
    hits = []
    for p in range(4):
        t = O.rw_boundaries(99, O.counter(tree, 0, 0, p, 0) >> 4, 16, lo, hi)
        if np.float32(t[root["bin"]]) == np.float32(root["threshold"]):
            hits.append(p)
    assert hits, "no keyed boundary matches the recorded threshold"
    left = int(np.sum(v < root["threshold"]))
    assert left == nodes[root["left"]]["n_samples"]


# --------------------------------------------------------------------------
# random-width bins (bin boundaries at random-width intervals)
# --------------------------------------------------------------------------

def test_rw_boundaries_sorted_in_range_and_unbiased():
    # The widths are i.i.d., so over many projections boundary i sits on
    # average at i/B of [lo, hi]; a slip in the prefix index (G_{i+1} for G_i)
    # moves every mean by 1/B, far outside the tolerance.
    for B in (2, 3, 16, 256):
        m = 3000
        acc = np.zeros(B - 1)
        for q in range(m):
            t = O.rw_boundaries(7, q, B, 0.0, 1.0)
            assert len(t) == B - 1
            assert np.all(np.diff(t) >= 0) and t[0] >= 0.0
            assert t[-1] <= np.nextafter(np.float32(1.0), np.float32(2.0))
            acc += t
        mean = acc / m
        want = np.arange(1, B) / B
        assert np.max(np.abs(mean - want)) < 0.4 / B, (B, np.max(np.abs(mean - want)))
    a = O.rw_boundaries(1, 5, 64, -2.0, 3.0)
    assert np.array_equal(a, O.rw_boundaries(1, 5, 64, -2.0, 3.0))
    assert not np.array_equal(a, O.rw_boundaries(2, 5, 64, -2.0, 3.0))
    assert not np.array_equal(a, O.rw_boundaries(1, 6, 64, -2.0, 3.0))


def test_rw_bin_is_upper_bound():
    rng = np.random.default_rng(77)
    for trial in range(200):
        B = int(rng.choice([2, 3, 5, 16, 64, 256]))
        lo, hi = sorted((rng.normal(size=2) * rng.choice([1e-3, 1.0, 1e3])).astype(np.float32).tolist())
        t = O.rw_boundaries(trial, 3 * trial, B, lo, hi)
        probe = np.concatenate([rng.uniform(lo, hi, 40).astype(np.float32), t,
                                np.nextafter(t, np.float32(-np.inf)), np.nextafter(t, np.float32(np.inf)),
                                np.array([lo, hi], np.float32)])
        tl = [float(x) for x in t]
        for v in probe:
            assert O.rw_bin(t, B, v) == bisect.bisect_right(tl, float(v))


@pytest.mark.parametrize("seed", range(60))
def test_rw_hist_path_matches_bruteforce(seed):
    # integer projected values (exact in FP32); the bins come from the oracle's
    # boundaries through bisect, the best split from exact rationals
    rng = np.random.default_rng(5000 + seed)
    n = int(rng.integers(2, 14))
    C = int(rng.integers(2, 5))
    d = 5
    Xi = rng.integers(-int(rng.choice([4, 1000])), 1001, size=(d, n))
    y = rng.integers(0, C, size=n).astype(np.int32)
    k = int(rng.integers(1, 5))
    B = int(rng.choice([2, 3, 4, 8, 16, 100, 256]))
    bseed = int(rng.integers(0, 2**63))
    feats, weights = random_projs(rng, k, d, 3)
    vals = exact_values(Xi, feats, weights, range(n))
    bins, bounds = [], []
    for p, vs in enumerate(vals):
        t = O.rw_boundaries(bseed, p, B, float(min(vs)), float(max(vs)))
        bounds.append(t)
        tl = [float(x) for x in t]
        bins.append([bisect.bisect_right(tl, float(v)) for v in vs])
    want = BF.best_bin_split(bins, y.tolist(), C, B)
    sp, H, _ = one_node(Xi.astype(np.float32), y, C, feats, weights, T=0, bins=B, hist=True,
                        bin_mode=O.BINS_RANDOM, bin_seed=bseed)
    assert sp["kind"] == 2
    for p in range(k):
        for b in range(B):
            for c in range(C):
                assert H[p, b, c] == sum(1 for kk, yy in zip(bins[p], y) if kk == b and yy == c)
    if want is None:
        assert sp["proj"] == -1 and sp["gain"] == 0.0
        return
    g, p, b, n_left = want
    assert (sp["proj"], sp["bin"], sp["n_left"]) == (p, b, n_left)
    assert sp["threshold"] == bounds[p][b]
    assert sum(1 for v in vals[p] if v < float(bounds[p][b])) == n_left
    assert abs(Fraction(float(sp["gain"])) - g) <= g * Fraction(1, 2**50)


def test_rw_partition_sends_values_below_the_threshold_left():
    rng = np.random.default_rng(91)
    d, n_rows = 10, 6000
    X = rng.standard_normal((d, n_rows)).astype(np.float32)
    y = rng.integers(0, 3, n_rows).astype(np.int32)
    sizes = [0, 1, 2, 5, 64, 300, 1000, 2500]
    offs = np.zeros(len(sizes) + 1, np.int32)
    offs[1:] = np.cumsum(sizes)
    idx = rng.permutation(n_rows)[:offs[-1]].astype(np.int32)
    k = 4
    po = (np.arange(len(sizes) + 1) * k).astype(np.int32)
    feats, weights = random_projs(rng, k * len(sizes), d, 3)
    zo = np.zeros(len(feats) + 1, np.int32)
    zo[1:] = np.cumsum([len(f) for f in feats])
    nf = np.concatenate([np.asarray(f, np.int32) for f in feats])
    nw = np.concatenate([np.asarray(w, np.int8) for w in weights])
    sp, _ = O.find_splits(X, y, 3, offs, idx, po, zo, nf, nw, bins=64, sort_threshold=0,
                          bin_mode=O.BINS_RANDOM, bin_seed=123)
    out, coff = O.partition(X, offs, idx, po, zo, nf, nw, sp, bins=64)
    for v in range(len(sizes)):
        a, b = offs[v], offs[v + 1]
        assert sp[v]["kind"] == 2
        if sp[v]["proj"] < 0:
            assert coff[2 * v + 1] == b
            continue
        q = po[v] + sp[v]["proj"]
        f, w = nf[zo[q]:zo[q + 1]], nw[zo[q]:zo[q + 1]]
        vals = np.array([O.project_value(X, f, w, r) for r in idx[a:b]], np.float32)
        left = idx[a:b][vals < sp[v]["threshold"]]
        right = idx[a:b][~(vals < sp[v]["threshold"])]
        assert coff[2 * v + 1] - a == sp[v]["n_left"] == left.size
        assert np.array_equal(out[a:b], np.concatenate([left, right]))


# --------------------------------------------------------------------------
# forest prediction
# --------------------------------------------------------------------------

def _small_forest(seed, n=1500, d=10, C=3, trees=3, T=40, max_depth=64):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((d, n)).astype(np.float32)
    y = rng.integers(0, C, n).astype(np.int32)
    roots = [np.sort(np.random.default_rng(seed * 10 + t).integers(0, n, n)).astype(np.int32)
             for t in range(trees)]
    ro = np.arange(trees + 1, dtype=np.int64) * n
    nodes, _, _ = O.grow_forest(X, y, C, ro, np.concatenate(roots), k=6, z=3, seed=seed, bins=64,
                                sort_threshold=T, max_depth=max_depth)
    root_ids = np.array([int(np.nonzero((nodes["depth"] == 0) & (nodes["tree"] == t))[0][0])
                         for t in range(trees)], np.int32)
    return X, y, C, roots, nodes, root_ids


def test_predict_routes_in_bag_samples_to_their_leaves():
    # the traversal rule must agree with the partition that grew the tree: the
    # in-bag samples of every tree reach each leaf exactly n_samples times
    X, y, C, roots, nodes, root_ids = _small_forest(11)
    for t, r in enumerate(root_ids):
        counts = {}
        for row in roots[t]:
            leaf = O.leaf_of(X, nodes, int(r), int(row))
            assert nodes[leaf]["is_leaf"] == 1 and nodes[leaf]["tree"] == t
            counts[leaf] = counts.get(leaf, 0) + 1
        leaves = np.nonzero((nodes["tree"] == t) & (nodes["is_leaf"] == 1))[0]
        for leaf in leaves:
            assert counts.get(int(leaf), 0) == nodes[leaf]["n_samples"], (t, leaf)


def test_predict_pure_tree_fits_in_bag_labels():
    X, y, C, roots, nodes, root_ids = _small_forest(12, trees=1, T=100)
    leaves = nodes[nodes["is_leaf"] == 1]
    votes, pred = O.predict(X, nodes, root_ids, C)
    inbag = np.unique(roots[0])
    # continuous features: every leaf of a tree grown to purity is pure
    assert np.array_equal(pred[inbag], y[inbag])
    assert np.all(votes.sum(axis=1) == 1) and leaves.size > 1


def test_predict_votes_and_majority():
    X, y, C, roots, nodes, root_ids = _small_forest(13, trees=5)
    votes, pred = O.predict(X, nodes, root_ids, C)
    assert np.all(votes.sum(axis=1) == 5)
    assert np.array_equal(pred, np.argmax(votes, axis=1))
    for t in range(5):
        one_v, one_p = O.predict(X, nodes, root_ids[t:t + 1], C)
        labels = np.array([nodes[O.leaf_of(X, nodes, int(root_ids[t]), r)]["label"] for r in range(0, 1500, 7)])
        assert np.array_equal(one_p[0:1500:7], labels)


# --------------------------------------------------------------------------
# entropy criterion
# --------------------------------------------------------------------------

def _ulp(x: float) -> float:
    return math.ulp(x) if x else math.ulp(1.0)


def test_ln_int_within_two_ulp_of_libm():
    ks = list(range(1, 5000)) + [2**e + d for e in range(1, 31) for d in (-1, 0, 1)]
    ks += [int(math.sqrt(2) * 2**e) + d for e in range(1, 30) for d in (-1, 0, 1)]
    ks += list(np.random.default_rng(3).integers(1, 2**31 - 1, 2000))
    for k in ks:
        k = int(k)
        if k < 1:
            continue
        got, want = O.ln_int(k), math.log(k)
        assert abs(got - want) <= 2 * _ulp(want), (k, got, want)


def _check_entropy_choice(sp, cands, n_tol=1e-12):
    """The oracle's pick is a best candidate up to rounding, and the unique one
    when it wins by a clear margin."""
    best = max((g for g, *_ in cands), default=None)
    if best is None or best <= n_tol:
        assert sp["proj"] == -1 and sp["gain"] == 0.0
        return
    assert sp["proj"] >= 0
    mine = [c for c in cands if (c[1], c[2]) == (sp["proj"], sp["bin"]) or
            (isinstance(c[2], float) and (c[1], c[3]) == (sp["proj"], sp["n_left"]))]
    assert mine, "the oracle's candidate is not one of the enumerated ones"
    assert abs(sp["gain"] - best) <= 1e-12 * max(1.0, best)
    assert mine[0][0] >= best - 1e-12
    ordered = sorted(cands, key=lambda c: -c[0])
    if len(ordered) == 1 or ordered[0][0] - ordered[1][0] > 1e-9:
        g, p, t, n_left = ordered[0]
        assert sp["proj"] == p and sp["n_left"] == n_left


@pytest.mark.parametrize("seed", range(60))
def test_entropy_hist_path_matches_bruteforce(seed):
    rng = np.random.default_rng(7000 + seed)
    n = int(rng.integers(2, 14))
    C = int(rng.integers(2, 5))
    d = 5
    Xi = rng.integers(-1000, 1001, size=(d, n))
    y = rng.integers(0, C, size=n).astype(np.int32)
    k = int(rng.integers(1, 5))
    B = int(rng.choice([2, 3, 8, 16, 100, 256]))
    feats, weights = random_projs(rng, k, d, 3)
    vals = exact_values(Xi, feats, weights, range(n))
    bins = []
    for vs in vals:
        lo, hi = min(vs), max(vs)
        row = []
        for v in vs:
            if hi == lo:
                row.append(0)
                continue
            e = Fraction(v - lo) * B / (hi - lo)
            if e < B and e != 0 and abs(e - round(e)) < Fraction(1, 10**5) * max(1, e):
                pytest.skip("a sample sits on a bin edge within rounding")
            row.append(min(math.floor(e), B - 1))
        bins.append(row)
    sp, _, _ = one_node(Xi.astype(np.float32), y, C, feats, weights, T=0, bins=B, criterion=O.CRIT_ENTROPY)
    cands = BF.all_bin_gains(bins, y.tolist(), C, B)
    _check_entropy_choice(sp, cands)
    if sp["proj"] >= 0:
        assert 0.0 < sp["gain"] <= BF.entropy(y.tolist(), C) + 1e-12


@pytest.mark.parametrize("seed", range(40))
def test_entropy_sort_path_matches_bruteforce(seed):
    rng = np.random.default_rng(8000 + seed)
    n = int(rng.integers(2, 14))
    C = int(rng.integers(2, 5))
    d = 5
    Xi = rng.integers(-3, 4, size=(d, n))
    y = rng.integers(0, C, size=n).astype(np.int32)
    k = int(rng.integers(1, 5))
    feats, weights = random_projs(rng, k, d, 3)
    vals = exact_values(Xi, feats, weights, range(n))
    sp, _, _ = one_node(Xi.astype(np.float32), y, C, feats, weights, T=1 << 30, criterion=O.CRIT_ENTROPY)
    cands = [(g, p, float(t), nl) for g, p, t, nl in BF.all_threshold_gains(vals, y.tolist(), C)]
    _check_entropy_choice(sp, cands)
