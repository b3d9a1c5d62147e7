"""GPU parity of forest prediction (sof_predict) with the oracle's traversal:
votes and predicted classes exactly equal, for forests grown by the oracle and
by the GPU, and for a random tree that mixes every split rule."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2603_00326_amd import sof as S
    return S.Context(0)


def gpu_predict(ctx, X, nodes, roots, C):
    import torch
    from paper_2603_00326_amd import sof as S
    Xd = torch.from_numpy(X).to("cuda:0")
    nd = S.nodes_to_device(nodes)
    rd = torch.from_numpy(np.asarray(roots, np.int32)).to("cuda:0")
    V, P = S.predict(ctx, Xd, nd, rd, C)
    torch.cuda.synchronize()
    return V.cpu().numpy(), P.cpu().numpy()


def check(ctx, X, nodes, roots, C, tag):
    say(f"[gpu] predict {tag}: rows={X.shape[1]} nodes={len(nodes)} trees={len(roots)} dtype={X.dtype}")
    v, p = gpu_predict(ctx, X, nodes, roots, C)
    wv, wp = O.predict(X, nodes, roots, C)
    assert np.array_equal(v, wv), f"{tag}: votes differ at rows {np.nonzero((v != wv).any(1))[0][:5]}"
    assert np.array_equal(p, wp), f"{tag}: predictions differ"


def test_predict_oracle_grown_forest(ctx):
    rng = np.random.default_rng(5)
    d, n, C, trees = 12, 3000, 3, 4
    X = rng.standard_normal((d, n)).astype(np.float32)
    y = rng.integers(0, C, n).astype(np.int32)
    roots = [np.sort(np.random.default_rng(60 + t).integers(0, n, n)).astype(np.int32) for t in range(trees)]
    ro = np.arange(trees + 1, dtype=np.int64) * n
    nodes, _, _ = O.grow_forest(X, y, C, ro, np.concatenate(roots), k=6, z=3, seed=9, bins=64,
                                sort_threshold=60, max_depth=64)
    check(ctx, X, nodes, np.arange(trees), C, "oracle forest, training rows")
    Xq = rng.standard_normal((d, 20000)).astype(np.float32)
    check(ctx, Xq, nodes, np.arange(trees), C, "oracle forest, new rows")


def test_predict_gpu_grown_forest_fp16(ctx):
    import torch
    from paper_2603_00326_amd import sof as S
    rng = np.random.default_rng(6)
    d, n, C, trees = 16, 4000, 4, 3
    grid = lambda m: (np.clip(np.rint(rng.standard_normal((d, m)) * 256.0), -2048, 2048) / 256.0)
    X = grid(n).astype(np.float16)
    y = rng.integers(0, C, n).astype(np.int32)
    ri = np.concatenate([np.sort(np.random.default_rng(70 + t).integers(0, n, n)) for t in range(trees)])
    f = S.Forest(ctx, torch.from_numpy(X).to("cuda:0"), torch.from_numpy(y).to("cuda:0"), C,
                 np.arange(trees + 1, dtype=np.int64) * n, torch.from_numpy(ri.astype(np.int32)).to("cuda:0"),
                 k=8, z=4, seed=3, bins=128, sort_threshold=100)
    f.grow()
    nodes = f.export()
    Xq = grid(30000).astype(np.float16)
    V, P = f.predict(torch.from_numpy(Xq).to("cuda:0"))
    torch.cuda.synchronize()
    f.close()
    wv, wp = O.predict(Xq, nodes, np.arange(trees), C)
    assert np.array_equal(V.cpu().numpy(), wv) and np.array_equal(P.cpu().numpy(), wp)


def random_tree(rng, d, C, depth, X):
    """A complete tree of the given depth with random rules of every kind."""
    nodes = np.zeros(2 ** (depth + 1) - 1, O.TREE_NODE_DTYPE)
    for i in range(len(nodes)):
        t = nodes[i]
        t["tree"], t["depth"] = 0, int(np.floor(np.log2(i + 1)))
        t["parent"] = (i - 1) // 2 if i else -1
        if 2 * i + 2 < len(nodes):
            t["is_leaf"], t["left"], t["right"] = 0, 2 * i + 1, 2 * i + 2
            z = int(rng.integers(1, 17))
            feats = np.sort(rng.choice(d, z, replace=False))
            w = rng.choice(np.array([-1, 1], np.int8), z)
            t["nnz"] = z
            t["feature"][:z] = feats
            t["weight"][:z] = w
            v = np.array([O.project_value(X, feats, w, r) for r in range(0, X.shape[1], 97)], np.float32)
            kind = int(rng.integers(0, 3))
            t["kind"] = kind
            if kind == 0:
                B = int(rng.choice([2, 16, 256]))
                lo, hi = float(v.min()), float(v.max())
                t["n_bins"], t["lo"], t["scale"] = B, lo, O.bin_scale(B, lo, hi)
                t["bin"] = int(rng.integers(0, B - 1))
            else:
                t["threshold"] = v[int(rng.integers(0, len(v)))]
                t["bin"] = -1
        else:
            t["is_leaf"], t["left"], t["right"], t["kind"] = 1, -1, -1, -1
            t["label"] = int(rng.integers(0, C))
    return nodes


@pytest.mark.parametrize("dt", [np.float32, np.float16])
def test_predict_random_tree_every_rule(ctx, dt):
    rng = np.random.default_rng(8)
    d, C = 24, 5
    X = (np.clip(np.rint(rng.standard_normal((d, 50000)) * 256.0), -2048, 2048) / 256.0).astype(dt)
    trees = [random_tree(rng, d, C, 7, X) for _ in range(3)]
    offs = np.cumsum([0] + [len(t) for t in trees])
    for t, o in zip(trees, offs):
        for f in ("left", "right", "parent"):
            t[f] = np.where(t[f] >= 0, t[f] + o, t[f])
        t["tree"] = int(np.searchsorted(offs, o))
    nodes = np.concatenate(trees)
    check(ctx, X, nodes, offs[:-1], C, f"random trees {np.dtype(dt).name}")


def test_predict_density_sampler_forest(ctx):
    # FP32 weights in the records: every internal node's projection rounds
    # each product, as the oracle's traversal does
    rng = np.random.default_rng(7)
    d, n, C, trees = 30, 3000, 3, 3
    X = rng.standard_normal((d, n)).astype(np.float32)
    y = rng.integers(0, C, n).astype(np.int32)
    roots = [np.sort(np.random.default_rng(80 + t).integers(0, n, n)).astype(np.int32) for t in range(trees)]
    ro = np.arange(trees + 1, dtype=np.int64) * n
    nodes, _, _ = O.grow_forest(X, y, C, ro, np.concatenate(roots), k=8, z=2, seed=11, bins=128,
                                sort_threshold=200, max_depth=64, sampler=O.SAMPLER_DENSITY,
                                weights=O.WEIGHTS_UNIFORM)
    assert len(set(nodes["nnz"][nodes["is_leaf"] == 0].tolist())) > 1
    Xq = rng.standard_normal((d, 20000)).astype(np.float32)
    check(ctx, Xq, nodes, np.arange(trees), C, "density-sampler forest, new rows")
