"""Seeded synthetic workloads for per-node split search.

This module only draws inputs: feature matrices, labels, frontiers and sparse
+/-1 projections.  It holds none of the split-search arithmetic, so both the
CPU oracle and the GPU library can consume its arrays without sharing any
code with each other.

Layout conventions (the C ABI uses the same ones):

* ``X`` has shape ``(d, n_rows)`` in C order, i.e. feature ``f`` of row ``r``
  is ``X[f, r]`` and every feature column is contiguous (column store).
* ``y`` is int32 in ``[0, n_classes)``.
* A frontier is ``node_offsets`` (int32, N+1) plus ``sample_idx`` (int32);
  node ``v`` owns ``sample_idx[node_offsets[v]:node_offsets[v+1]]``.
* Projections are CSR: ``proj_offsets`` (int32, N+1) maps a node to its range
  of projections, ``nz_offsets`` (int32, P+1) maps a projection to its range of
  nonzeros, ``nz_feature`` (int32, ascending within a projection, distinct) and
  ``nz_weight`` (int8 +/-1, or FP32 weights: ``with_float_weights``).

The paper measures on HIGGS, SUSY, Epsilon and Trunk; none is available here,
so these generators stand in for them with dense real-valued column stores of
similar shape (1M-row and >=1K-feature scales, 2-4 classes).
"""
from __future__ import annotations

import concurrent.futures as _cf
import os
from dataclasses import dataclass, field

import numpy as np

INT32_MAX = 2**31 - 1

_POOL_WORKERS = max(1, min(16, os.cpu_count() or 1))


@dataclass
class Workload:
    """One batch of split-search input (host arrays)."""

    name: str
    X: np.ndarray                 # (d, n_rows) float32 or float16, C order
    y: np.ndarray                 # (n_rows,) int32
    n_classes: int
    node_offsets: np.ndarray      # (N+1,) int32
    sample_idx: np.ndarray        # (total,) int32
    proj_offsets: np.ndarray      # (N+1,) int32
    nz_offsets: np.ndarray        # (P+1,) int32
    nz_feature: np.ndarray        # (nnz,) int32
    nz_weight: np.ndarray         # (nnz,) int8 +/-1, or FP32 weights
    bins: int = 256
    sort_threshold: int = 0
    node_bins: np.ndarray | None = None   # (N,) int32 or None
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.node_offsets.shape[0] - 1)

    @property
    def n_samples(self) -> int:
        return int(self.node_offsets[-1])

    @property
    def n_proj(self) -> int:
        return int(self.proj_offsets[-1])

    @property
    def units(self) -> int:
        """Node-sample x projection units: sum over nodes of n_v * k_v."""
        n = np.diff(self.node_offsets.astype(np.int64))
        k = np.diff(self.proj_offsets.astype(np.int64))
        return int((n * k).sum())

    @property
    def max_proj_per_node(self) -> int:
        k = np.diff(self.proj_offsets)
        return int(k.max()) if k.size else 0


# ----------------------------------------------------------------------------
# column generation (one independent PCG64 stream per feature, so the result
# does not depend on how many threads fill it)
# ----------------------------------------------------------------------------

def _fill_columns(d: int, n: int, seed: int, fill, dtype=np.float32) -> np.ndarray:
    X = np.empty((d, n), dtype=dtype)
    seqs = np.random.SeedSequence(seed).spawn(d)

    def work(f):
        rng = np.random.Generator(np.random.PCG64(seqs[f]))
        X[f, :] = fill(f, rng, n)

    if d * n >= 1 << 22:
        with _cf.ThreadPoolExecutor(_POOL_WORKERS) as ex:
            list(ex.map(work, range(d)))
    else:
        for f in range(d):
            work(f)
    return X


def _normal_fill(f, rng, n):
    return rng.standard_normal(n, dtype=np.float32)


def _flip_labels(rng: np.random.Generator, y: np.ndarray, p: float, n_classes: int) -> np.ndarray:
    """Replace each label with probability p by a uniformly drawn *other* class."""
    y = y.astype(np.int32, copy=True)
    flip = rng.random(y.shape[0]) < p
    if n_classes == 2:
        y[flip] = 1 - y[flip]
    else:
        shift = rng.integers(1, n_classes, size=int(flip.sum()), dtype=np.int32)
        y[flip] = (y[flip] + shift) % n_classes
    return y


def _sparse_scores(rng, X, n_scores, nnz, d):
    """Scores s_c = sum_j w_j x_j over nnz random distinct features (float64)."""
    n = X.shape[1]
    s = np.zeros((n_scores, n), dtype=np.float64)
    for c in range(n_scores):
        feats = rng.choice(d, size=nnz, replace=False)
        w = rng.choice(np.array([-1.0, 1.0]), size=nnz)
        for f, wf in zip(feats, w):
            s[c] += wf * X[f].astype(np.float64)
    return s


def random_projections(rng: np.random.Generator, n_nodes: int, k: int, d: int,
                       z, *, z_max: int | None = None):
    """CSR projections: k per node, each of z distinct ascending features with +/-1 weights.

    ``z`` is an int, or a tuple ``(lo, hi)`` for a per-projection uniform draw of
    the nonzero count in ``[lo, hi]``.
    """
    P = n_nodes * k
    if isinstance(z, tuple):
        zs = rng.integers(z[0], z[1] + 1, size=P).astype(np.int32)
    else:
        zs = np.full(P, int(z), dtype=np.int32)
    nz_offsets = np.zeros(P + 1, dtype=np.int32)
    np.cumsum(zs, out=nz_offsets[1:])
    nnz = int(nz_offsets[-1])
    nz_feature = np.empty(nnz, dtype=np.int32)
    # distinct features per projection: argpartition of uniform keys is slow for
    # large d; draw with rejection of duplicates instead (z << d).
    zmax = int(zs.max()) if P else 0
    cand = rng.integers(0, d, size=(P, max(zmax * 2, 1)), dtype=np.int32)
    for q in range(P):
        zq = int(zs[q])
        if zq == 0:
            continue
        row = cand[q]
        seen = []
        for c in row:
            if c not in seen:
                seen.append(int(c))
                if len(seen) == zq:
                    break
        while len(seen) < zq:
            c = int(rng.integers(0, d))
            if c not in seen:
                seen.append(c)
        seen.sort()
        nz_feature[nz_offsets[q]:nz_offsets[q + 1]] = seen
    nz_weight = rng.choice(np.array([-1, 1], dtype=np.int8), size=nnz)
    proj_offsets = (np.arange(n_nodes + 1, dtype=np.int64) * k).astype(np.int32)
    return proj_offsets, nz_offsets, nz_feature, nz_weight


def uniform_weights(rng: np.random.Generator, n: int) -> np.ndarray:
    """n FP32 weights (2m + 1 - 2^24) / 2^24, m uniform on 0..2^24-1: symmetric
    on (-1, 1), never 0, each exactly representable."""
    m = rng.integers(0, 1 << 24, size=n, dtype=np.int64)
    return ((2 * m + 1 - (1 << 24)).astype(np.float64) / float(1 << 24)).astype(np.float32)


def with_float_weights(wl: "Workload", seed: int) -> "Workload":
    """The same workload with FP32 weights from uniform_weights in place of +/-1."""
    wl.nz_weight = uniform_weights(np.random.default_rng(seed), len(wl.nz_feature))
    return wl


def _random_projections_fast(rng, n_nodes, k, d, z):
    """Vectorised variant of random_projections for fixed z (same distribution)."""
    P = n_nodes * k
    feats = np.empty((P, z), dtype=np.int32)
    todo = np.arange(P)
    while todo.size:
        draw = rng.integers(0, d, size=(todo.size, z), dtype=np.int32)
        s = np.sort(draw, axis=1)
        ok = np.all(s[:, 1:] != s[:, :-1], axis=1) if z > 1 else np.ones(todo.size, bool)
        feats[todo[ok]] = s[ok]
        todo = todo[~ok]
    nz_feature = feats.reshape(-1)
    nz_weight = rng.choice(np.array([-1, 1], dtype=np.int8), size=P * z)
    nz_offsets = (np.arange(P + 1, dtype=np.int64) * z).astype(np.int32)
    proj_offsets = (np.arange(n_nodes + 1, dtype=np.int64) * k).astype(np.int32)
    return proj_offsets, nz_offsets, nz_feature, nz_weight


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def config1(sort: bool = False, seed: int = 0) -> Workload:
    """Single root node: n=4096, d=64 N(0,1), y=[x0+x2-x5>0] with 10% flips,
    k=64 projections of 3 distinct features, 256 bins.  ``sort`` picks the
    all-sort run (threshold INT32_MAX) instead of the all-histogram run (0)."""
    n, d, k, z = 4096, 64, 64, 3
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((d, n), dtype=np.float32)
    s = X[0].astype(np.float64) + X[2].astype(np.float64) - X[5].astype(np.float64)
    y = _flip_labels(rng, (s > 0).astype(np.int32), 0.10, 2)
    po, no, nf, nw = random_projections(rng, 1, k, d, z)
    return Workload("c1_root_4096x64" + ("_sort" if sort else "_hist"), X, y, 2,
                    np.array([0, n], np.int32), np.arange(n, dtype=np.int32),
                    po, no, nf, nw, bins=256,
                    sort_threshold=INT32_MAX if sort else 0,
                    meta=dict(config=1, k=k, z=z, d=d))


def accuracy_data(seed: int = 7, n_train: int = 4096, n_test: int = 100_000, d: int = 64):
    """Training and held-out rows from config 1's rule: d N(0,1) features,
    y = [x0 + x2 - x5 > 0] with 10% of labels flipped (both sets)."""
    rng = np.random.default_rng(seed)
    out = []
    for n in (n_train, n_test):
        X = rng.standard_normal((d, n), dtype=np.float32)
        s = X[0].astype(np.float64) + X[2].astype(np.float64) - X[5].astype(np.float64)
        out += [X, _flip_labels(rng, (s > 0).astype(np.int32), 0.10, 2)]
    return tuple(out)


def config2(seed: int = 1, n: int = 1 << 20) -> Workload:
    """Root node at scale: n=2^20, d=256 (128 N(0,1) + 128 Bernoulli(0.1)),
    2 classes from a random 6-feature oblique rule with 5% flips, k=256, z=3."""
    d, k, z = 256, 256, 3

    def fill(f, rng, m):
        if f < 128:
            return rng.standard_normal(m, dtype=np.float32)
        return (rng.random(m) < 0.1).astype(np.float32)

    X = _fill_columns(d, n, seed, fill)
    rng = np.random.default_rng([seed, 7])
    S = rng.choice(d, size=6, replace=False)
    w = rng.choice(np.array([-1.0, 1.0]), size=6)
    mu = np.where(S < 128, 0.0, 0.1)
    s = np.zeros(n, np.float64)
    for f, wf in zip(S, w):
        s += wf * X[f].astype(np.float64)
    y = _flip_labels(rng, (s > float(np.sum(w * mu))).astype(np.int32), 0.05, 2)
    po, no, nf, nw = _random_projections_fast(rng, 1, k, d, z)
    return Workload("c2_root_1Mx256", X, y, 2, np.array([0, n], np.int32),
                    np.arange(n, dtype=np.int32), po, no, nf, nw, bins=256,
                    sort_threshold=0, meta=dict(config=2, k=k, z=z, d=d))


def config3_sizes(seed: int = 2, n_nodes: int = 4096) -> np.ndarray:
    rng = np.random.default_rng([seed, 1])
    eps = rng.standard_normal(n_nodes)
    return np.clip(np.rint(np.exp(np.log(300.0) + 1.55 * eps)), 2, 100000).astype(np.int32)


def config3(layout: str = "a", seed: int = 2, n_nodes: int = 4096, d: int = 512,
            scale_rows: float = 1.0) -> Workload:
    """Batched frontier: 4096 log-normal nodes (median 300, clipped 2..100000,
    ~4M samples) over a shared N(0,1) matrix with d=512, 3 classes, k=64
    projections per node of 4 nonzeros.  Layout ``a``: node v owns a contiguous
    row range; layout ``b``: each node's rows are an ascending random subset."""
    sizes = config3_sizes(seed, n_nodes)
    if scale_rows != 1.0:
        sizes = np.maximum(2, np.rint(sizes * scale_rows)).astype(np.int32)
    n_rows = int(sizes.sum())
    X = _fill_columns(d, n_rows, seed, _normal_fill)
    rng = np.random.default_rng([seed, 2])
    s = _sparse_scores(rng, X, 3, 4, d)
    y = _flip_labels(rng, np.argmax(s, axis=0).astype(np.int32), 0.05, 3)
    offs = np.zeros(n_nodes + 1, np.int64)
    np.cumsum(sizes, out=offs[1:])
    if layout == "a":
        idx = np.arange(n_rows, dtype=np.int32)
    elif layout == "b":
        perm = rng.permutation(n_rows).astype(np.int32)
        idx = np.empty(n_rows, np.int32)
        for v in range(n_nodes):
            idx[offs[v]:offs[v + 1]] = np.sort(perm[offs[v]:offs[v + 1]])
    else:
        raise ValueError(layout)
    po, no, nf, nw = _random_projections_fast(rng, n_nodes, 64, d, 4)
    return Workload(f"c3{layout}_frontier4096_d{d}", X, y, 3, offs.astype(np.int32), idx,
                    po, no, nf, nw, bins=256, sort_threshold=0,
                    meta=dict(config=3, layout=layout, k=64, z=4, d=d))


def config4_data(seed: int = 4, n: int = 2_000_000, d: int = 1024, n_trees: int = 8):
    """Full-training input: n rows, d features (90% exact zeros, rest N(0,1)),
    4 classes from argmax of 4 random +/-1 scores over 32 features, 5% flips,
    and one bootstrap root per tree (n draws with replacement, sorted)."""

    def fill(f, rng, m):
        col = np.zeros(m, np.float32)
        mask = rng.random(m) < 0.1
        col[mask] = rng.standard_normal(int(mask.sum()), dtype=np.float32)
        return col

    X = _fill_columns(d, n, seed, fill)
    rng = np.random.default_rng([seed, 3])
    s = _sparse_scores(rng, X, 4, 32, d)
    y = _flip_labels(rng, np.argmax(s, axis=0).astype(np.int32), 0.05, 4)
    roots = [np.sort(np.random.default_rng(seed + t).integers(0, n, n)).astype(np.int32)
             for t in range(n_trees)]
    root_offsets = np.zeros(n_trees + 1, np.int64)
    np.cumsum([r.size for r in roots], out=root_offsets[1:])
    return X, y, 4, root_offsets, np.concatenate(roots) if roots else np.zeros(0, np.int32)


def grid_matrix(seed: int, n: int, d: int) -> np.ndarray:
    """Features N(0, variance 2) rounded half-to-even to multiples of 1/256 and
    clipped to [-8, 8]; every value is exact in FP16 and FP32."""

    def fill(f, rng, m):
        v = rng.standard_normal(m) * np.sqrt(2.0)
        return (np.clip(np.rint(v * 256.0), -2048, 2048) / 256.0).astype(np.float32)

    return _fill_columns(d, n, seed, fill)


def config5(seed: int = 5, n: int = 10_000_000, fp16: bool = True) -> Workload:
    """Reduced-precision storage: n=10M, d=128 grid features stored FP16 (or the
    identical FP32 values), 2 classes, k=128 projections with 1..8 nonzeros."""
    d, k = 128, 128
    X32 = grid_matrix(seed, n, d)
    rng = np.random.default_rng([seed, 5])
    S = rng.choice(d, size=6, replace=False)
    w = rng.choice(np.array([-1.0, 1.0]), size=6)
    s = np.zeros(n, np.float64)
    for f, wf in zip(S, w):
        s += wf * X32[f].astype(np.float64)
    y = _flip_labels(rng, (s > 0).astype(np.int32), 0.05, 2)
    po, no, nf, nw = random_projections(rng, 1, k, d, (1, 8))
    X = X32.astype(np.float16) if fp16 else X32
    return Workload("c5_root_10Mx128_" + ("f16" if fp16 else "f32"), X, y, 2,
                    np.array([0, n], np.int32), np.arange(n, dtype=np.int32),
                    po, no, nf, nw, bins=256, sort_threshold=0,
                    meta=dict(config=5, k=k, d=d))


def sub_frontier(wl: Workload, nodes) -> Workload:
    """The frontier restricted to the given nodes, in the given order (same
    matrix and labels; each node keeps its samples and projections)."""
    no = wl.node_offsets.astype(np.int64)
    po = wl.proj_offsets.astype(np.int64)
    zo = wl.nz_offsets.astype(np.int64)
    idx, offs, pof, zof, zf, zw = [], [0], [0], [0], [], []
    for v in nodes:
        idx.append(wl.sample_idx[no[v]:no[v + 1]])
        offs.append(offs[-1] + int(no[v + 1] - no[v]))
        zf.append(wl.nz_feature[zo[po[v]]:zo[po[v + 1]]])
        zw.append(wl.nz_weight[zo[po[v]]:zo[po[v + 1]]])
        z = np.diff(zo[po[v]:po[v + 1] + 1])
        zof.extend((zof[-1] + np.cumsum(z)).tolist())
        pof.append(pof[-1] + int(po[v + 1] - po[v]))
    cat = lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt)
    nb = None if wl.node_bins is None else wl.node_bins[np.asarray(nodes, np.int64)].astype(np.int32)
    return Workload(wl.name + "_sample", wl.X, wl.y, wl.n_classes, np.asarray(offs, np.int32),
                    cat(idx, np.int32), np.asarray(pof, np.int32), np.asarray(zof, np.int32),
                    cat(zf, np.int32), cat(zw, np.int8), wl.bins, wl.sort_threshold, nb, dict(wl.meta))


# ----------------------------------------------------------------------------
# small random frontiers for parity tests
# ----------------------------------------------------------------------------

def random_frontier(seed: int, *, n_rows: int, d: int, n_classes: int, sizes,
                    k: int, z, bins: int = 256, sort_threshold: int = 0,
                    layout: str = "b", integer_features: int | None = None,
                    dtype=np.float32, node_bins=None) -> Workload:
    """A frontier over a shared matrix with given node sizes.

    ``integer_features`` draws features as small integers in
    ``[-integer_features, integer_features]`` (many ties); otherwise N(0,1).
    ``layout`` ``a`` gives contiguous row ranges (needs sum(sizes) <= n_rows),
    ``b`` ascending random subsets, ``r`` random order with repeats allowed.
    """
    rng = np.random.default_rng(seed)
    sizes = np.asarray(sizes, dtype=np.int64)
    if integer_features is not None:
        X = rng.integers(-integer_features, integer_features + 1, size=(d, n_rows)).astype(np.float32)
    else:
        X = rng.standard_normal((d, n_rows), dtype=np.float32)
    if dtype == np.float16:
        X = (np.rint(X * 256.0) / 256.0).clip(-8, 8).astype(np.float16)
    y = rng.integers(0, n_classes, size=n_rows).astype(np.int32)
    offs = np.zeros(sizes.size + 1, np.int64)
    np.cumsum(sizes, out=offs[1:])
    parts = []
    for v, m in enumerate(sizes):
        m = int(m)
        if layout == "a":
            parts.append(np.arange(offs[v], offs[v] + m, dtype=np.int32))
        elif layout == "b":
            parts.append(np.sort(rng.choice(n_rows, size=m, replace=False)).astype(np.int32))
        else:
            parts.append(rng.integers(0, n_rows, size=m).astype(np.int32))
    idx = np.concatenate(parts) if parts else np.zeros(0, np.int32)
    po, no, nf, nw = random_projections(rng, sizes.size, k, d, z)
    nb = None
    if node_bins is not None:
        nb = np.asarray(node_bins, dtype=np.int32)
    return Workload(f"random_frontier_{seed}", X, y, n_classes, offs.astype(np.int32), idx,
                    po, no, nf, nw, bins=bins, sort_threshold=sort_threshold, node_bins=nb)
