"""ctypes wrapper of the reference CPU implementation (``sof_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The GPU library never imports this module and
this module never imports the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "sof_oracle.c")]

SORT_LIMIT = 8192

SPLIT_DTYPE = np.dtype([
    ("proj", "<i4"), ("kind", "<i4"), ("bin", "<i4"), ("threshold", "<f4"),
    ("lo", "<f4"), ("scale", "<f4"), ("n_left", "<i4"), ("n_right", "<i4"),
    ("flags", "<i4"), ("pad", "<i4"), ("gain", "<f8"),
])
assert SPLIT_DTYPE.itemsize == 48

TREE_NODE_DTYPE = np.dtype([
    ("tree", "<i4"), ("depth", "<i4"), ("parent", "<i4"), ("left", "<i4"), ("right", "<i4"),
    ("n_samples", "<i4"), ("label", "<i4"), ("is_leaf", "<i4"), ("kind", "<i4"), ("bin", "<i4"),
    ("threshold", "<f4"), ("lo", "<f4"), ("scale", "<f4"), ("n_bins", "<i4"), ("nnz", "<i4"),
    ("pad", "<i4"), ("feature", "<i4", (16,)), ("weight", "<f4", (16,)), ("gain", "<f8"),
])
assert TREE_NODE_DTYPE.itemsize == 200


def build(force: bool = True) -> str:
    """Compile liboracle.so with plain IEEE binary32 semantics."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", LIB_PATH + ".tmp", *SOURCES, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        L.or_half_to_float.argtypes = [ctypes.c_uint16]
        L.or_half_to_float.restype = ctypes.c_float
        L.or_project_value.argtypes = [P, ctypes.c_int, i64, P, P, ctypes.c_int, i32]
        L.or_project_value.restype = ctypes.c_float
        L.or_bin_scale.argtypes = [ctypes.c_int, ctypes.c_float, ctypes.c_float]
        L.or_bin_scale.restype = ctypes.c_float
        L.or_bin_index.argtypes = [ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int]
        L.or_bin_index.restype = ctypes.c_int
        L.or_project.argtypes = [P, ctypes.c_int, i64, i32, P, P, P, P, P, P, P]
        L.or_project.restype = None
        L.or_find_splits.argtypes = [P, ctypes.c_int, i64, P, i32, i32, P, P, P, P, P, P, P, i32, i32,
                                     i32, u64, i32, P, P, i32]
        L.or_ln_int.argtypes = [i64]
        L.or_ln_int.restype = ctypes.c_double
        L.or_klnk.argtypes = [i64]
        L.or_klnk.restype = ctypes.c_double
        L.or_rw_boundaries.argtypes = [u64, i64, ctypes.c_int, ctypes.c_float, ctypes.c_float, P]
        L.or_rw_boundaries.restype = None
        L.or_rw_bin.argtypes = [P, ctypes.c_int, ctypes.c_float]
        L.or_rw_bin.restype = ctypes.c_int
        L.or_find_splits.restype = ctypes.c_int
        L.or_partition.argtypes = [P, ctypes.c_int, i64, i32, P, P, P, P, P, P, P, i32, P, P, P]
        L.or_partition.restype = None
        L.or_mix64.argtypes = [u64]
        L.or_mix64.restype = u64
        L.or_hash.argtypes = [u64, u64]
        L.or_hash.restype = u64
        L.or_counter.argtypes = [i32, i32, i32, i32, i32]
        L.or_counter.restype = u64
        L.or_sample_projection.argtypes = [u64, i32, i32, i32, i32, i32, i32, i32, i32, P, P]
        L.or_sample_projection.restype = i32
        L.or_density_nnz.argtypes = [u64, i32, i32, i32, i32, i32, i32]
        L.or_density_nnz.restype = i32
        L.or_sample_weight.argtypes = [u64, i32, i32, i32, i32, i32, i32, i32]
        L.or_sample_weight.restype = ctypes.c_float
        L.or_grow_forest.argtypes = [P, ctypes.c_int, i64, i32, P, i32, i32, i32, P, P, i32, i32, i32, i32, u64,
                                     i32, i32, i32, i32, i32, u64, i32, P, i64, P, P]
        L.or_grow_forest.restype = i64
        L.or_leaf_of.argtypes = [P, ctypes.c_int, i64, P, i32, i32]
        L.or_leaf_of.restype = i32
        L.or_predict.argtypes = [P, ctypes.c_int, i64, P, P, i32, i32, i32, P, P]
        L.or_predict.restype = None
        _lib = L
    return _lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def _xinfo(X):
    X = np.ascontiguousarray(X)
    if X.dtype == np.float16:
        return X, 1
    if X.dtype == np.float32:
        return X, 0
    raise TypeError(f"features must be float32 or float16, got {X.dtype}")


def half_to_float(h: int) -> float:
    return lib().or_half_to_float(int(h))


def bin_scale(n_bins: int, lo, hi) -> np.float32:
    return np.float32(lib().or_bin_scale(int(n_bins), float(lo), float(hi)))


def bin_index(v, lo, scale, n_bins: int) -> int:
    return int(lib().or_bin_index(float(v), float(lo), float(scale), int(n_bins)))


def project_value(X, feat, w, row) -> np.float32:
    X, dt = _xinfo(X)
    feat = _c(feat, np.int32)
    w = _c(w, np.float32)
    return np.float32(lib().or_project_value(_p(X), dt, X.shape[1], _p(feat), _p(w), len(feat), int(row)))


def project(X, node_offsets, sample_idx, proj_offsets, nz_offsets, nz_feature, nz_weight):
    X, dt = _xinfo(X)
    no, si, po = _c(node_offsets, np.int32), _c(sample_idx, np.int32), _c(proj_offsets, np.int32)
    zo, zf, zw = _c(nz_offsets, np.int32), _c(nz_feature, np.int32), _c(nz_weight, np.float32)
    n = np.diff(no.astype(np.int64))
    k = np.diff(po.astype(np.int64))
    out = np.empty(int((n * k).sum()), np.float32)
    lib().or_project(_p(X), dt, X.shape[1], len(no) - 1, _p(no), _p(si), _p(po), _p(zo), _p(zf), _p(zw),
                     _p(out))
    return out


BINS_EQUAL, BINS_RANDOM = 0, 1
CRIT_GINI, CRIT_ENTROPY = 0, 1


def ln_int(k: int) -> float:
    return float(lib().or_ln_int(int(k)))


def rw_boundaries(seed: int, q: int, n_bins: int, lo, hi) -> np.ndarray:
    """Random-width boundaries t[0..n_bins-2] of projection q."""
    t = np.zeros(max(n_bins - 1, 1), np.float32)
    lib().or_rw_boundaries(int(seed) & (2**64 - 1), int(q), int(n_bins), float(lo), float(hi), _p(t))
    return t[:n_bins - 1]


def rw_bin(t, n_bins: int, v) -> int:
    t = _c(t, np.float32)
    return int(lib().or_rw_bin(_p(t), int(n_bins), float(v)))


def find_splits(X, y, n_classes, node_offsets, sample_idx, proj_offsets, nz_offsets, nz_feature,
                nz_weight, *, bins=256, sort_threshold=0, node_bins=None, hist=False, threads=0,
                bin_mode=BINS_EQUAL, bin_seed=0, criterion=CRIT_GINI):
    """Best split per node.  Returns (splits[N] of SPLIT_DTYPE, hist or None)."""
    X, dt = _xinfo(X)
    y = _c(y, np.int32)
    no, si, po = _c(node_offsets, np.int32), _c(sample_idx, np.int32), _c(proj_offsets, np.int32)
    zo, zf, zw = _c(nz_offsets, np.int32), _c(nz_feature, np.int32), _c(nz_weight, np.float32)
    nb = _c(node_bins, np.int32)
    N = len(no) - 1
    P = int(po[-1])
    out = np.zeros(N, SPLIT_DTYPE)
    H = np.zeros((P, bins, n_classes), np.int32) if hist else None
    lib().or_find_splits(_p(X), dt, X.shape[1], _p(y), int(n_classes), N, _p(no), _p(si), _p(po), _p(zo),
                         _p(zf), _p(zw), _p(nb), int(bins), int(sort_threshold), int(bin_mode),
                         int(bin_seed) & (2**64 - 1), int(criterion), _p(out), _p(H), int(threads))
    return out, H


def find_splits_w(wl, **kw):
    """find_splits on a workload object (attributes as in the workload generators)."""
    kw.setdefault("bins", wl.bins)
    kw.setdefault("sort_threshold", wl.sort_threshold)
    kw.setdefault("node_bins", wl.node_bins)
    return find_splits(wl.X, wl.y, wl.n_classes, wl.node_offsets, wl.sample_idx, wl.proj_offsets,
                       wl.nz_offsets, wl.nz_feature, wl.nz_weight, **kw)


def partition(X, node_offsets, sample_idx, proj_offsets, nz_offsets, nz_feature, nz_weight, splits,
              *, bins=256, node_bins=None):
    X, dt = _xinfo(X)
    no, si, po = _c(node_offsets, np.int32), _c(sample_idx, np.int32), _c(proj_offsets, np.int32)
    zo, zf, zw = _c(nz_offsets, np.int32), _c(nz_feature, np.int32), _c(nz_weight, np.float32)
    nb = _c(node_bins, np.int32)
    sp = np.ascontiguousarray(splits, dtype=SPLIT_DTYPE)
    N = len(no) - 1
    out = np.empty_like(si)
    coff = np.empty(2 * N + 1, np.int32)
    lib().or_partition(_p(X), dt, X.shape[1], N, _p(no), _p(si), _p(po), _p(zo), _p(zf), _p(zw), _p(nb),
                       int(bins), _p(sp), _p(out), _p(coff))
    return out, coff


def mix64(z: int) -> int:
    return int(lib().or_mix64(z & (2**64 - 1)))


def hash64(seed: int, counter: int) -> int:
    return int(lib().or_hash(seed & (2**64 - 1), counter & (2**64 - 1)))


def counter(tree, level, pos, proj, draw) -> int:
    return int(lib().or_counter(tree, level, pos, proj, draw))


SAMPLER_FIXED, SAMPLER_DENSITY = 0, 1
WEIGHTS_SIGN, WEIGHTS_UNIFORM = 0, 1
SEED_NNZ, SEED_WEIGHT = 0x6A09E667F3BCC909, 0xBB67AE8584CAA73B   # streams of the density sampler


def sample_projection(seed, tree, level, pos, proj, n_features, z, sampler=SAMPLER_FIXED, weights=WEIGHTS_SIGN):
    """Features (ascending, int32) and FP32 weights of one drawn projection."""
    f = np.zeros(16, np.int32)
    w = np.zeros(16, np.float32)
    nz = lib().or_sample_projection(seed & (2**64 - 1), tree, level, pos, proj, n_features, sampler, z, weights,
                                    _p(f), _p(w))
    return f[:nz].copy(), w[:nz].copy()


def density_nnz(seed, tree, level, pos, proj, n_features, z) -> int:
    return int(lib().or_density_nnz(seed & (2**64 - 1), tree, level, pos, proj, n_features, z))


def sample_weight(seed, sampler, weights, tree, level, pos, proj, rank) -> np.float32:
    return np.float32(lib().or_sample_weight(seed & (2**64 - 1), sampler, weights, tree, level, pos, proj, rank))


def grow_forest(X, y, n_classes, root_offsets, root_idx, *, k, z, seed, bins=256, sort_threshold=0,
                max_depth=64, threads=0, cap=None, first_tree=0, sampler=SAMPLER_FIXED, weights=WEIGHTS_SIGN,
                criterion=CRIT_GINI, bin_mode=BINS_EQUAL, bin_seed=0):
    """Grow several trees level by level to purity.  Returns (nodes, level_nodes, level_units)."""
    X, dt = _xinfo(X)
    y = _c(y, np.int32)
    ro = _c(root_offsets, np.int64)
    ri = _c(root_idx, np.int32)
    n_trees = len(ro) - 1
    if cap is None:
        cap = max(16, 2 * int(ro[-1]) + n_trees)
    nodes = np.zeros(cap, TREE_NODE_DTYPE)
    ln = np.zeros(max_depth + 1, np.int64)
    lu = np.zeros(max_depth + 1, np.int64)
    n = lib().or_grow_forest(_p(X), dt, X.shape[1], X.shape[0], _p(y), int(n_classes), n_trees,
                             int(first_tree), _p(ro),
                             _p(ri), int(k), int(z), int(sampler), int(weights), seed & (2**64 - 1), int(bins),
                             int(sort_threshold),
                             int(max_depth), int(criterion), int(bin_mode), int(bin_seed) & (2**64 - 1),
                             int(threads), _p(nodes), int(cap), _p(ln), _p(lu))
    if n < 0:
        raise RuntimeError("node capacity too small")
    levels = int(np.count_nonzero(ln))
    return nodes[:n].copy(), ln[:levels].copy(), lu[:levels].copy()


def leaf_of(X, nodes, root: int, row: int) -> int:
    """Index of the leaf that row reaches from node root."""
    X, dt = _xinfo(X)
    nodes = np.ascontiguousarray(nodes, dtype=TREE_NODE_DTYPE)
    return int(lib().or_leaf_of(_p(X), dt, X.shape[1], _p(nodes), int(root), int(row)))


def predict(X, nodes, roots, n_classes: int):
    """Forest prediction for every row of X: (votes (n_rows, C) int32, pred (n_rows,) int32)."""
    X, dt = _xinfo(X)
    nodes = np.ascontiguousarray(nodes, dtype=TREE_NODE_DTYPE)
    roots = _c(roots, np.int32)
    n = X.shape[1]
    votes = np.zeros((n, n_classes), np.int32)
    pred = np.zeros(n, np.int32)
    lib().or_predict(_p(X), dt, X.shape[1], _p(nodes), _p(roots), len(roots), int(n_classes), n, _p(votes),
                     _p(pred))
    return votes, pred
